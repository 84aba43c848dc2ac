#!/usr/bin/env python3
"""Benchmark: GEM pixel-frame updates per second on one MI355X.

Workload: one synthetic street window at 1216x352 with N = 6 flows, K = 32 depth candidates
per pixel per pass and 10 GEM iterations (random initial depth, perturbed initial poses).
One step = the whole window: initial depth, 10 iterations (coarse pass, local pass, pose
step) and the final E-step / confidence / statistics.  Inputs are resident in device memory
before the timed region.  The unit of work is one (reference pixel, frame) pair carried
through one GEM iteration: 1216 * 352 * 6 * 10 = 25.68 M units per window.

Also reported, on the same JSON line:
  roofline      the dominant kernel (the fused local-level E+M pass): its launches inside the
                timed steps are bracketed with HIP events on their launch stream by the
                library's timers; achieved = algorithmic FP32 flops per launch / average
                launch duration, against the FP32 vector ALU peak.  traffic = HBM-side bytes
                per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary committed under
                profiles/ (null when the library sources changed since it was taken);
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same window (GEM iteration 0
                on the full image), timed on this host;
  batch         64 uneven windows (320..1216 x 240..352, N 3..8, half with a depth prior),
                10 iterations each: 64 sequential whole-window calls against one replay of
                the batched launch sequence captured in a HIP graph (windows/s, per-window
                latency percentiles);
  learned_init  plain GEM against GEM started from the learned proposal on held-out
                640x480 windows: median error, and ms to reach plain GEM's median error;
  proposal      the proposal network's forward pass at 640x480 (BF16 implicit-GEMM
                convolutions on the matrix cores) against the dense BF16 peak.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--only-window]
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU work of one local-level pass per (pixel, frame), counted as the survey of
# the method does: K candidate evaluations of ~48 lane-op slots each (reprojection,
# bilinear flow sample, residual, log-logistic MIE cost; a transcendental counts 4) plus
# ~55 slots for the E-step's emission and forward-backward at the current value.
SLOTS_PER_CAND_FRAME = 48.0
SLOTS_ESTEP_PER_PIXEL_FRAME = 55.0
# Unpacked FP32 vector issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-op slots/s
# (packed FP32, which doubles it to the published 157.3 TFLOP/s, is not emitted).
PEAK_VALU_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_BF16_TFLOPS = 2500.0           # dense BF16 matrix-core peak
# stored (computed) channel counts of the proposal network's layers: (c_in, c_out, scale)
PROPOSAL_LAYERS = [(16, 64, 1), (64, 128, 0.25), (128, 128, 0.25), (128, 128, 0.25), (128, 64, 1), (64, 32, 1)]
# Algorithmic bytes of one local-level launch per pixel: per frame the flow (8 B) and the
# rigidness written (4 B); inverse depth read and written (8 B); the coarse value (4 B per
# lattice cell of s*s = 16 pixels).
BYTES_PER_PIXEL_FRAME = 12.0
BYTES_PER_PIXEL = 8.0 + 4.0 / 16
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_level_local_1216x352_n6_k32_hbm_bytes.txt")


# the sources the local-level kernel is compiled from
LEVEL_SOURCES = ("device.h", "kernels.h", "gem_kernels.hip")


def source_hash():
    h = hashlib.sha256()
    for f in LEVEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_06800_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM-side bytes per launch of the local-level kernel from the committed counter summary,
    or None when it is absent or was taken on other library sources."""
    try:
        rows = dict(l.split(":", 1) for l in open(TRAFFIC_SUMMARY) if ":" in l and not l.startswith(" "))
        if rows["source_sha256_16"].strip() != source_hash():
            return None
        return float(rows["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-window", action="store_true", help="skip the batch / learned-init / proposal parts")
    ap.add_argument("--only-batch", action="store_true",
                    help="only the 64-window batch, its windows generated in this process (for profilers)")
    ap.add_argument("--only-proposal", action="store_true",
                    help="only the proposal network's forward pass at 640x480 (for profilers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the windows of a batch are "
              "independent and would shard across GPUs without communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 512 * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 512 MiB three times")
        return

    from paper_2104_06800_amd import synth
    from paper_2104_06800_amd.binding import TIMER_COARSE, TIMER_LOCAL, TIMER_POSE, Voldor

    if args.only_proposal:
        from paper_2104_06800_amd import proposal as pr
        lib = Voldor(0)
        params, _ = pr.load(os.path.join(ROOT, "paper_2104_06800_amd", "weights", "proposal_n6.npz"))
        net = lib.net_alloc(params)
        print(json.dumps({"proposal": proposal_forward_workload(lib, torch, net, synth.make_window(4, 10 ** 6),
                                                                params=params)}), flush=True)
        lib.close()
        return

    if args.only_batch:
        lib = Voldor(0)
        print(json.dumps({"batch": batch_workload(lib, np, torch, args, pool=False)}), flush=True)
        lib.close()
        return

    t0 = time.time()
    w = synth.make_window(2, 0)
    p = w["params"]
    H, W, N, K, I = p["H"], p["W"], p["N"], p["n_candidates"], p["iters"]
    log(f"workload generated in {time.time() - t0:.1f}s: {W}x{H} N={N} K={K} iters={I}")

    lib = Voldor(0)
    b = lib.alloc(p, w["flow"], w["pose_init"])
    pose0 = b["pose"].clone()

    def step():
        b["pose"].copy_(pose0)
        lib.run(p, b, iters=I)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # only the dominant kernel's launches are bracketed in the timed steps: every event
    # record adds a few microseconds to the stream
    lib.timing(True, timers=(TIMER_LOCAL,))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    local_timer = lib.timing_read(TIMER_LOCAL)
    # per-phase breakdown from separate windows with every class bracketed
    n_split = 2
    lib.timing(True)
    for _ in range(n_split):
        step()
    torch.cuda.synchronize()
    split = {name: lib.timing_read(t) for name, t in (("local", TIMER_LOCAL), ("coarse", TIMER_COARSE),
                                                       ("pose", TIMER_POSE))}
    lib.timing(False)
    units = H * W * N * I
    value = units / (ms / 1e3)
    stats = b["stats"].cpu().numpy()
    rho = b["idepth"].cpu().numpy()
    static = ~w["dynamic"]
    err = np.abs(rho - w["idepth_gt"]) / w["idepth_gt"]
    from paper_2104_06800_amd.proposal import median_rel_error
    log(f"window: {ms:.3f} ms  ->  {value / 1e9:.3f} G pixel-frame updates/s; median static inverse-depth "
        f"rel error {np.median(err[static]):.4f} (after median scaling "
        f"{median_rel_error(rho, w['idepth_gt'], static):.4f}); loglik {stats[0]:.6g}")
    per_window = {k: v[0] * 1e3 / n_split for k, v in split.items()}
    log("per window (separate windows, every timer class on): " +
        ", ".join(f"{k} {v:.0f} us ({split[k][1] // n_split} brackets)" for k, v in per_window.items()))

    # dominant kernel: the fused local-level pass, every launch of it in the timed steps
    k_ms_total, k_n = local_timer
    k_ms = k_ms_total / k_n
    slots = H * W * N * (K * SLOTS_PER_CAND_FRAME + SLOTS_ESTEP_PER_PIXEL_FRAME)
    alg_bytes = H * W * (N * BYTES_PER_PIXEL_FRAME + BYTES_PER_PIXEL)
    achieved = slots / (k_ms / 1e3) / 1e12
    traffic = measured_traffic()
    log(f"local level pass: {k_ms * 1e3:.1f} us/launch over {k_n} launches, {slots / 1e9:.2f} G VALU slots "
        f"algorithmic, {achieved:.2f} T slots/s; algorithmic bytes {alg_bytes / 1e6:.1f} MB "
        f"({alg_bytes / (k_ms / 1e3) / 1e9:.0f} GB/s); counted traffic "
        f"{'n/a' if traffic is None else f'{traffic / 1e6:.1f} MB'}")
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TSLOTS, 2),
                "unit": "T VALU lane-op slots/s", "frac": round(achieved / PEAK_VALU_TSLOTS, 4),
                "traffic": None if traffic is None else round(traffic),
                "traffic_unit": "bytes per launch (FETCH_SIZE x 2 + WRITE_SIZE)",
                "algorithmic_bytes": round(alg_bytes), "kernel": "k_level (local level, fused E+M)",
                "kernel_us": round(k_ms * 1e3, 2), "launches": k_n,
                "window_us": {k: round(v, 1) for k, v in per_window.items()}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, H, W, N, K)

    extra = {}
    if not args.only_window:
        extra["vc"] = vc_workload(lib, np, torch, w, b)
        extra["pose_sample"] = pose_sample_workload(lib, np, torch, w, b)
        extra["hierarchy"] = hierarchy_sweep(lib, np, torch, w)
        extra["batch"] = batch_workload(lib, np, torch, args)
        extra["learned_init"], extra["proposal"] = learned_init(lib, np, torch)
        extra["align"] = align_workload(lib, np, torch)
        extra["sim3"] = sim3_workload(lib, np, torch)
        extra["keyframe"] = keyframe_workload(lib, np, torch)

    out = {
        "metric": "GEM pixel-frame updates/s at 1216x352 N=6",
        "value": round(value, 1),
        "unit": "pixel-frame updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "street window 1216x352, N=6 flows, K=32 candidates, 10 GEM iterations",
                   "H": H, "W": W, "N": N, "K": K, "iters": I, "tile": p["tile"],
                   "coarse_stride": p["coarse_stride"], "pose_gn_steps": p["pose_gn_steps"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)
    lib.close()


def _oracle_iteration(w):
    """GEM iteration 0 of a window by the FP64 oracle, single-threaded; returns seconds."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import gem as ogem
    p = w["params"]
    ob = ogem.alloc_buffers(p, w["flow"], w["pose_init"])
    ogem.init_idepth(p, ob)
    t0 = time.perf_counter()
    ogem.gem_step(p, ob, 0)
    return time.perf_counter() - t0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, H, W, N, K):
    """The FP64 oracle as it stands on this host: GEM iteration 0 of the benchmark window on one
    core, then the same iteration of independent copies of the window on every core of the
    GPU's host share at once (windows are independent, so that is the oracle's throughput on
    all cores)."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    cs1 = _oracle_iteration(w)
    one = H * W * N / cs1
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        per = list(ex.map(_oracle_iteration, [w] * cores))
    wall = time.perf_counter() - t0
    allc = cores * H * W * N / max(per)
    log(f"oracle: {cs1:.1f} s for one iteration on one core -> {one:.0f} pixel-frame updates/s; "
        f"{cores} cores at once: {max(per):.1f} s each (wall {wall:.1f} s) -> {allc:.0f}")
    return {"value": round(allc, 1), "unit": "pixel-frame updates/s", "cores": cores, "kind": "oracle",
            "value_one_core": round(one, 1), "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"GEM iteration 0 of the same {W}x{H} N={N} K={K} window (FP64 numpy): once on one "
                      f"core ({cs1:.1f} s), then {cores} independent copies at once, one per core "
                      f"({max(per):.1f} s)"}


def _pool_generate(fn, items, workers=16):
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, items))


ALIGN_BYTES_PER_PIXEL_STEP = 16     # map-2 inverse depth + confidence, map-1 plane sample


def _align_pairs(seed):
    from paper_2104_06800_amd import synth
    return synth.make_pairs(1, H=480, W=640, seed=seed, noise_rel=0.01, conf="random")


def align_workload(lib, np, torch, n_pairs=32, reps=5):
    """Keyframe point-to-plane alignment of n_pairs 640x480 inverse-depth map pairs in one
    call (10 Gauss-Newton steps each, identity start): time per call and pose error against
    the ground truth."""
    from scipy.spatial.transform import Rotation
    t0 = time.time()
    prs = _pool_generate(_align_pairs, [3_400_000 + i for i in range(n_pairs)])
    ap = prs[0]["params"]
    cat = lambda k: np.concatenate([p[k] for p in prs])
    dev = torch.device("cuda", 0)
    t = lambda a, dt=torch.float32: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    r1, r2, c2 = t(cat("idepth1")), t(cat("idepth2")), t(cat("conf2"))
    gt = cat("pose_gt")
    log(f"align: {n_pairs} pairs generated in {time.time() - t0:.1f}s")
    pose = torch.zeros((n_pairs, 6), dtype=torch.float64, device=dev)
    lib.align_p2p(ap, r1, r2, c2, pose)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        pose.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, status = lib.align_p2p(ap, r1, r2, c2, pose)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    got = pose.cpu().numpy()
    rot_err = [np.degrees((Rotation.from_rotvec(g[:3]) * Rotation.from_rotvec(x[:3]).inv()).magnitude())
               for g, x in zip(got, gt)]
    tr_err = np.linalg.norm(got[:, 3:] - gt[:, 3:], axis=1)
    steps = ap["gn_steps"]
    px_steps = n_pairs * ap["H"] * ap["W"] * steps
    out = {"pairs": n_pairs, "H": ap["H"], "W": ap["W"], "gn_steps": steps, "ms_per_call": round(ms, 3),
           "pairs_per_s": round(n_pairs / (ms / 1e3), 1),
           "algorithmic_GB_per_s": round(px_steps * ALIGN_BYTES_PER_PIXEL_STEP / (ms / 1e3) / 1e9, 1),
           "median_rot_err_deg": round(float(np.median(rot_err)), 5),
           "median_trans_err": round(float(np.median(tr_err)), 6),
           "converged": int((status.cpu().numpy() == 0).sum()),
           "workload": "synthetic room pairs, motion <= 2 deg / 0.1, 1% inverse-depth noise, random confidence"}
    log("align: " + json.dumps(out))
    return out


def pose_sample_workload(lib, np, torch, w, b, reps=10):
    """The paper's sampled pose M-step on the street window's GEM output: 256 q-weighted P3P
    samples per frame, meanshift mode and 3-sigma covariance fit for frames 1..N, one call;
    time per call and the poses' distance to the truth before and after."""
    from scipy.spatial.transform import Rotation
    p = w["params"]
    sp = dict(samples=256, tries=16, sigma_w=0.01, sigma_t_rel=0.02, eps=1e-12)
    pose0 = b["pose"].clone()
    lib.rigidness_fb(p, b, p["iters"], 1)
    lib.pose_sample(p, b, p["iters"], sp)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        b["pose"].copy_(pose0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, info = lib.pose_sample(p, b, p["iters"], sp)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    got, gt, start = b["pose"].cpu().numpy(), w["pose_gt"], pose0.cpu().numpy()
    b["pose"].copy_(pose0)
    rot = lambda a: float(np.median([np.degrees((Rotation.from_rotvec(x[:3]) * Rotation.from_rotvec(y[:3]).inv()).magnitude())
                                     for x, y in zip(a, gt)]))
    out = {"ms_per_call": round(float(np.median(ts)), 3), "frames": p["N"], "samples_per_frame": sp["samples"],
           "median_rot_err_deg_before": round(rot(start), 4), "median_rot_err_deg_after": round(rot(got), 4),
           "valid_samples_frame1": int(info.cpu().numpy()[0, 0]),
           "workload": "street window 1216x352 N=6 after 10 GEM iterations (GEM's Gauss-Newton poses as the start)"}
    log("pose sample: " + json.dumps(out))
    return out


def sim3_workload(lib, np, torch, n_pairs=32, reps=5):
    """7-DoF keyframe alignment (motion and relative depth scale, Levenberg-Marquardt, 15
    evaluations) of the synthetic 640x480 pairs with map 1 scaled by a known factor."""
    prs = _pool_generate(_align_pairs, [3_400_000 + i for i in range(n_pairs)])
    ap = dict(prs[0]["params"], gn_steps=15)
    cat = lambda k: np.concatenate([p[k] for p in prs])
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(3)
    s_true = rng.uniform(0.7, 1.4, n_pairs)
    t = lambda a, dt=torch.float32: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
    r1 = t(cat("idepth1") * s_true[:, None, None].astype(np.float32))
    r2, c2 = t(cat("idepth2")), t(cat("conf2"))
    gt = cat("pose_gt")
    from paper_2104_06800_amd import synth
    start = np.stack([synth.vo_start(rng, x, 1.0, 0.02) for x in gt])
    pose = torch.as_tensor(start, dtype=torch.float64, device=dev)
    scale = torch.ones(n_pairs, dtype=torch.float64, device=dev)
    ts = []
    for _ in range(reps + 1):
        pose.copy_(torch.as_tensor(start, dtype=torch.float64))
        scale.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, status = lib.align_sim3(ap, r1, r2, c2, pose, scale)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    got_s = scale.cpu().numpy()
    out = {"pairs": n_pairs, "H": ap["H"], "W": ap["W"], "evaluations": ap["gn_steps"],
           "ms_per_call": round(float(np.median(ts[1:])), 3),
           "median_scale_rel_err": round(float(np.median(np.abs(got_s / s_true - 1))), 6),
           "median_pose_err": round(float(np.median(np.abs(pose.cpu().numpy() - gt).max(1))), 6),
           "converged": int((status.cpu().numpy() == 0).sum()),
           "workload": "synthetic room pairs as in align, map 1 scaled by U[0.7, 1.4], start within 1 deg / 2 cm, s = 1"}
    log("sim3: " + json.dumps(out))
    return out


def _keyframe_pair(k):
    from paper_2104_06800_amd import synth
    return synth.keyframe_pair(k)


def keyframe_workload(lib, np, torch, n_pairs=32, reps=5):
    """The prior-window workload: 2 x n_pairs indoor 640x480, N=8 windows with one depth prior
    each (ground truth with 5% multiplicative noise and 10% holes, 6-DoF motion <= 5 deg /
    0.3 m), GEM on each (timed per window), then the n_pairs keyframe alignments on the GEM
    outputs and window b's confidence in one call: Huber delta 0.02, 10 Gauss-Newton steps,
    started from the chained visual-odometry estimate (the true relative pose moved by up to
    1 deg and 3 cm per axis)."""
    from scipy.spatial.transform import Rotation
    from paper_2104_06800_amd import synth
    t0 = time.time()
    pairs = _pool_generate(_keyframe_pair, list(range(n_pairs)))
    log(f"keyframe: {n_pairs} pairs ({2 * n_pairs} prior windows) generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    maps1, maps2, confs, errs, win_ms = [], [], [], [], []
    for wa, wb, _ in pairs:
        for w, tgt in ((wa, "a"), (wb, "b")):
            p = w["params"]
            b = lib.alloc(p, w["flow"], w["pose_init"], w["prior_idepth"], w["prior_pose"])
            pose0 = b["pose"].clone()
            lib.run(p, b, iters=p["iters"])            # warm-up (and the result: runs are deterministic)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b["pose"].copy_(pose0)
            e0.record()
            lib.run(p, b, iters=p["iters"])
            e1.record()
            torch.cuda.synchronize()
            win_ms.append(e0.elapsed_time(e1))
            rho = b["idepth"].cpu().numpy()
            errs.append(float(np.median(np.abs(rho - w["idepth_gt"]) / w["idepth_gt"])))
            if tgt == "a":
                maps1.append(rho)
            else:
                maps2.append(rho)
                confs.append(b["conf"].cpu().numpy())
            del b
    p = pairs[0][0]["params"]
    H, W, N, I = p["H"], p["W"], p["N"], p["iters"]
    fx, fy, cx, cy = pairs[0][0]["intr"]
    ap = dict(H=H, W=W, fx=fx, fy=fy, cx=cx, cy=cy, robust=0, robust_scale=0.02, gn_steps=10,
              normal_disc_rel=0.2, scale_s=1.0)
    rng = np.random.default_rng(11)
    truth = np.stack([pr[2] for pr in pairs])
    start = np.stack([synth.vo_start(rng, x) for x in truth])
    t = lambda a, dt=torch.float32: torch.as_tensor(np.stack(a), dtype=dt, device=dev).contiguous()
    r1, r2, c2 = t(maps1), t(maps2), t(confs)
    pose = torch.as_tensor(start, dtype=torch.float64, device=dev)
    lib.align_p2p(ap, r1, r2, c2, pose)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        pose.copy_(torch.as_tensor(start, dtype=torch.float64))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, st, status = lib.align_p2p(ap, r1, r2, c2, pose)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    got = pose.cpu().numpy()
    rot_err = lambda a, b: [np.degrees((Rotation.from_rotvec(g[:3]) * Rotation.from_rotvec(x[:3]).inv()).magnitude())
                            for g, x in zip(a, b)]
    ms_w = float(np.median(win_ms))
    out = {"windows": 2 * n_pairs, "H": H, "W": W, "N": N, "iters": I, "P": 1,
           "window_ms_p50": round(ms_w, 3), "window_ms_p90": round(float(np.percentile(win_ms, 90)), 3),
           "window_updates_per_s": round(H * W * N * I / (ms_w / 1e3), 1),
           "median_window_rel_error": round(float(np.median(errs)), 4),
           "align_ms_per_call": round(float(np.median(ts)), 3), "align_pairs": n_pairs,
           "align_median_rot_err_deg": round(float(np.median(rot_err(got, truth))), 4),
           "align_median_trans_err": round(float(np.median(np.linalg.norm(got[:, 3:] - truth[:, 3:], axis=1))), 5),
           "start_median_rot_err_deg": round(float(np.median(rot_err(start, truth))), 4),
           "start_median_trans_err": round(float(np.median(np.linalg.norm(start[:, 3:] - truth[:, 3:], axis=1))), 5),
           "align_converged": int((status.cpu().numpy() == 0).sum()),
           "workload": "indoor room windows 640x480 N=8 with a 5%-noise depth prior (10% holes), GEM from "
                       "the prior, then keyframe alignment of the GEM outputs and confidence (Huber 0.02, "
                       "10 Gauss-Newton steps, from a visual-odometry start within 1 deg / 3 cm)"}
    log("keyframe: " + json.dumps(out))
    return out
def batch_workload(lib, np, torch, args, pool=True):
    from paper_2104_06800_amd import synth
    t0 = time.time()
    specs = synth.batch_shapes()
    if pool:
        wins = _pool_generate(synth.batch_window, specs)
    else:
        wins = []
        for i, sp in enumerate(specs):
            wins.append(synth.batch_window(sp))
            if i % 8 == 7:
                log(f"batch: {i + 1} of {len(specs)} windows generated")
    log(f"batch: {len(wins)} windows generated in {time.time() - t0:.1f}s")
    items = []
    for w in wins:
        p = w["params"]
        b = lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))
        items.append((p, b, b["pose"].clone()))
    iters = items[0][0]["iters"]
    assert all(p["iters"] == iters for p, _, _ in items)

    def reset():
        for _, b, p0 in items:
            b["pose"].copy_(p0)

    # sequential whole-window calls, each timed with events on the current stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in items]
    for rep in range(2):
        reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for (p, b, _), (e0, e1) in zip(items, ev):
            e0.record()
            lib.run(p, b, iters=iters)
            e1.record()
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t1) * 1e3
    per = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    # batched: the first call captures the graph, later identical calls replay it
    batch = [(p, b) for p, b, _ in items]
    reset()
    lib.batch_run(batch, iters)
    torch.cuda.synchronize()
    reps = 5
    ts = []
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.batch_run(batch, iters)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t1) * 1e3)
    bat_ms = float(np.median(ts))
    px = sum(p["H"] * p["W"] * p["N"] for p, _, _ in items) * iters
    log(f"batch: sequential {seq_ms:.2f} ms ({len(items) / seq_ms * 1e3:.0f} windows/s), batched graph "
        f"{bat_ms:.2f} ms ({len(items) / bat_ms * 1e3:.0f} windows/s)")
    from paper_2104_06800_amd.proposal import median_rel_error
    keys = ("idepth", "rigid", "pose", "conf", "stats")
    fixed_out = [{k: b[k].clone() for k in keys} for _, b, _ in items]
    err_plain = [median_rel_error(b["idepth"].cpu().numpy(), w["idepth_gt"], ~w["dynamic"])
                 for (_, b, _), w in zip(items, wins)]

    def timed_batch(fn, reps=5):
        out = []
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t1) * 1e3)
        return float(np.median(out))

    # autotuned knobs per window shape (coordinate descent; results must not change)
    from paper_2104_06800_amd import autotune
    t0 = time.time()
    space = dict(local_chains=(2, 4, 8), local_spec=(1, 2, 3), coarse_spec=(4, 6, 8), local_order=(1, 2))
    table = {}
    for w in wins:
        table[autotune.bucket(w["params"])] = autotune.tune(lib, w, reps=2, space=space)
    tune_s = time.time() - t0
    lib.batch_run(batch, iters)                  # recapture with the tuned knobs
    tuned_ms = timed_batch(lambda: lib.batch_run(batch, iters))
    same = all(torch.equal(b[k], f[k]) for (_, b, _), f in zip(items, fixed_out) for k in keys)
    ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in items]
    reset()
    for (p, b, _), (e0, e1) in zip(items, ev2):
        e0.record()
        lib.run(p, b, iters=iters)
        e1.record()
    torch.cuda.synchronize()
    per_tuned = np.array([e0.elapsed_time(e1) for e0, e1 in ev2])
    for w in wins:
        lib.set_knobs(w["params"], None)
    log(f"batch: autotuned ({tune_s:.0f} s of tuning) batched graph {tuned_ms:.2f} ms against {bat_ms:.2f} ms "
        f"fixed; sequential per-window sum {per_tuned.sum():.2f} against {per.sum():.2f} ms; results identical: {same}")
    # learned start in the batch: the proposal network's start of every window, captured in
    # the same graph, and fewer iterations
    from paper_2104_06800_amd import proposal as pr
    params, _ = pr.load(os.path.join(ROOT, "paper_2104_06800_amd", "weights", "proposal_n6.npz"))
    net = lib.net_alloc(params)
    learned = {}
    for k_it in (iters, 8):
        reset()
        fbs = torch.zeros(len(items), dtype=torch.int32, device="cuda")
        lib.batch_run_learned(net, batch, k_it, fallback=fbs)
        l_ms = timed_batch(lambda: lib.batch_run_learned(net, batch, k_it, fallback=fbs))
        errs = [median_rel_error(b["idepth"].cpu().numpy(), w["idepth_gt"], ~w["dynamic"])
                for (_, b, _), w in zip(items, wins)]
        learned[k_it] = {"batched_graph_ms": round(l_ms, 3), "windows_per_s": round(len(items) / l_ms * 1e3, 1),
                         "median_window_error": round(float(np.median(errs)), 4),
                         "fallbacks": int(fbs.sum().cpu())}
        log(f"batch: learned start, {k_it} iterations: {l_ms:.2f} ms, median window error "
            f"{np.median(errs):.4f} (plain {np.median(err_plain):.4f}), fallbacks {int(fbs.sum().cpu())}")
    return {"windows": len(items), "iters": iters, "pixel_frame_updates": px,
            "autotuned": {"batched_graph_ms": round(tuned_ms, 3), "fixed_batched_graph_ms": round(bat_ms, 3),
                          "sequential_sum_ms": round(float(per_tuned.sum()), 3),
                          "fixed_sequential_sum_ms": round(float(per.sum()), 3),
                          "results_identical": bool(same), "tuning_s": round(tune_s, 1),
                          "buckets": len(table), "space": {k: list(v) for k, v in space.items()},
                          "per_window_ms_sequential": {q: round(float(np.percentile(per_tuned, int(q[1:]))), 3)
                                                       for q in ("p50", "p90", "p99")}},
            "learned_start": {"median_window_error_plain": round(float(np.median(err_plain)), 4),
                              **{f"iters_{k}": v for k, v in learned.items()}},
            "sequential_ms": round(seq_ms, 3), "batched_graph_ms": round(bat_ms, 3),
            "windows_per_s_sequential": round(len(items) / seq_ms * 1e3, 1),
            "windows_per_s_batched": round(len(items) / bat_ms * 1e3, 1),
            "speedup": round(seq_ms / bat_ms, 3),
            "per_window_ms_sequential": {"p50": round(float(np.percentile(per, 50)), 3),
                                         "p90": round(float(np.percentile(per, 90)), 3),
                                         "p99": round(float(np.percentile(per, 99)), 3)},
            "per_window_ms_batched": {"p50": round(bat_ms, 3), "p90": round(bat_ms, 3), "p99": round(bat_ms, 3),
                                      "note": "every window of a replay completes with its last launch"},
            "shapes": "W 320..1216, H 240..352 (steps of 16), N 3..8, odd windows with a depth prior"}


def _psnr(rho, gt, static):
    """Depth-map quality as in the paper's runtime / quality plot: PSNR of the inverse depth
    against the ground truth over static pixels, after median scaling (monocular gauge).  The
    peak is the ground truth's 99th-percentile inverse depth, and each pixel's error is
    clipped at a tenth of it, so that the few gross outliers of moving-object boundaries do
    not decide the figure."""
    import numpy as np
    ok = static & np.isfinite(rho) & (rho > 0)
    s = np.median(gt[ok] / rho[ok])
    peak = np.percentile(gt[ok], 99)
    err = np.minimum(np.abs(rho[ok] * s - gt[ok]), 0.1 * peak)
    return float(10 * np.log10(peak ** 2 / np.mean(err ** 2)))


def hierarchy_sweep(lib, np, torch, w, reps=3):
    """Runtime against depth quality over the hierarchy's settings on the benchmark window:
    coarse stride s (s = 1: full-resolution lattice rows / columns, the global propagation
    of the method the paper builds on) and local tile T.  Each setting runs the full
    10-iteration window; its coarse passes and local passes are timed separately by the
    library's timers in extra windows."""
    from paper_2104_06800_amd.binding import TIMER_COARSE, TIMER_LOCAL
    from paper_2104_06800_amd.proposal import median_rel_error
    static = ~w["dynamic"]
    out = []
    for s, T in ((1, 256), (1, 32), (2, 32), (4, 16), (4, 32), (4, 64), (8, 32), (8, 64), (16, 64)):
        p = dict(w["params"], coarse_stride=s, tile=T)
        b = lib.alloc(p, w["flow"], w["pose_init"])
        pose0 = b["pose"].clone()

        def run():
            b["pose"].copy_(pose0)
            lib.run(p, b, iters=p["iters"])

        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        lib.timing(True, timers=(TIMER_LOCAL, TIMER_COARSE))
        run()
        torch.cuda.synchronize()
        coarse_ms, _ = lib.timing_read(TIMER_COARSE)
        local_ms, _ = lib.timing_read(TIMER_LOCAL)
        lib.timing(False)
        rho = b["idepth"].cpu().numpy()
        row = {"s": s, "T": T, "ms": round(float(np.median(ts)), 3), "coarse_ms": round(coarse_ms, 3),
               "local_ms": round(local_ms, 3), "psnr_db": round(_psnr(rho, w["idepth_gt"], static), 2),
               "median_static_rel_error": round(median_rel_error(rho, w["idepth_gt"], static), 4)}
        log("hierarchy: " + json.dumps(row))
        out.append(row)
        del b
    return out


def vc_workload(lib, np, torch, w, b, reps=20):
    """Visibility-coverage scores of the window's estimated inverse depth (confidence >= 0.5)
    against its N frames' estimated poses and a keyframe pose, in one call, with the first
    frame whose VC falls below tau_stride = 0.7."""
    from paper_2104_06800_amd.binding import VC_OUT_LEN  # noqa: F401  (ABI constant present)
    p = w["params"]
    vp = dict(H=p["H"], W=p["W"], fx=p["fx"], fy=p["fy"], cx=p["cx"], cy=p["cy"], cell=8, conf_min=0.5)
    poses = torch.cat([b["pose"], torch.tensor([[0.0, 0.03, 0.0, 0.2, 0.0, -12.0]], dtype=torch.float64,
                                               device=b["pose"].device)]).contiguous()
    out, first = lib.vc_scores(vp, b["idepth"], b["conf"], poses, 0.7)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lib.vc_scores(vp, b["idepth"], b["conf"], poses, 0.7)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    o = out.cpu().numpy()
    n = poses.shape[0]
    alg = p["H"] * p["W"] * 8          # inverse depth + confidence, read once for all poses
    res = {"us_per_call": round(us, 2), "poses": n, "vc": [round(float(x), 4) for x in o[:, 2]],
           "visibility": [round(float(x), 4) for x in o[:, 0]], "coverage": [round(float(x), 4) for x in o[:, 1]],
           "first_below_tau_0.7": int(first.cpu()[0]), "cell": 8,
           "algorithmic_GB_per_s": round(alg / (us * 1e-6) / 1e9, 1),
           "workload": f"{p['W']}x{p['H']} GEM output against its {n - 1} frames and one keyframe"}
    log("vc: " + json.dumps(res))
    return res


def proposal_forward_workload(lib, torch, net, w, reps=20, params=None):
    """MFMA throughput of the whole proposal network on one window's flows (inference), and
    with params the time of one training step (forward, loss, backward, Adam) on it."""
    from paper_2104_06800_amd import proposal as pr
    p = w["params"]
    H, W, N = p["H"], p["W"], p["N"]
    flow = lib.alloc(p, w["flow"], w["pose_init"])["flow"]
    tn = pr.tnorm_of(w["pose_init"])
    for _ in range(3):
        lib.proposal_forward(net, flow, tn, p["idepth_min"], p["idepth_max"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lib.proposal_forward(net, flow, tn, p["idepth_min"], p["idepth_max"])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # real channels: 2N flow components in, 1 + N heads out; the stored layers pad them to
    # 16 and 32 (the matrix-core tiles compute the padding too)
    real = [(2 * N if i == 0 else ci, 1 + N if i == len(PROPOSAL_LAYERS) - 1 else co, sc)
            for i, (ci, co, sc) in enumerate(PROPOSAL_LAYERS)]
    flops = sum(2.0 * H * W * sc * co * 9 * ci for ci, co, sc in real)
    flops_stored = sum(2.0 * H * W * sc * co * 9 * ci for ci, co, sc in PROPOSAL_LAYERS)
    achieved = flops / (ms / 1e3) / 1e12
    log(f"proposal forward at {W}x{H}: {ms:.3f} ms, {flops / 1e9:.1f} GFLOP on real channels "
        f"({flops_stored / 1e9:.1f} stored), {achieved:.1f} TFLOP/s")
    train_ms = None
    if params is not None:
        tnet = lib.net_alloc(params, train=True)
        rho_t = torch.full((H, W), 0.1, dtype=torch.float32, device=flow.device)
        q_t = torch.full((N, H, W), 0.9, dtype=torch.float32, device=flow.device)
        mask = torch.ones((H, W), dtype=torch.uint8, device=flow.device)
        loss = torch.zeros(3, dtype=torch.float64, device=flow.device)
        step = lambda k: lib.proposal_train_step(tnet, flow, tn, rho_t, q_t, mask, 0.5, 1e-5, k, loss)
        for k in range(3):
            step(k + 1)
        torch.cuda.synchronize()
        e0.record()
        for k in range(reps):
            step(k + 4)
        e1.record()
        torch.cuda.synchronize()
        train_ms = e0.elapsed_time(e1) / reps
        log(f"proposal training step at {W}x{H}: {train_ms:.3f} ms")
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "ms": round(ms, 4), "gflop": round(flops / 1e9, 2),
            "gflop_stored": round(flops_stored / 1e9, 2),
            "frac_stored": round(flops_stored / (ms / 1e3) / 1e12 / PEAK_BF16_TFLOPS, 4),
            "train_step_ms": None if train_ms is None else round(train_ms, 3),
            "workload": f"proposal forward {W}x{H}, N={N}, BF16 weights/activations, FP32 accumulation"}


def learned_init(lib, np, torch):
    from paper_2104_06800_amd import proposal as pr
    path = os.path.join(ROOT, "paper_2104_06800_amd", "weights", "proposal_n6.npz")
    params, meta = pr.load(path)
    net = lib.net_alloc(params)
    t0 = time.time()
    test = pr.generate(list(range(pr.TEST_SEED0, pr.TEST_SEED0 + 16)), 16)
    log(f"learned init: {len(test)} held-out windows generated in {time.time() - t0:.1f}s")
    res = pr.compare(lib, net, test, warm=False)
    summ = pr.summarize(res)
    log("learned init: " + json.dumps(summ))
    prop = proposal_forward_workload(lib, torch, net, test[0], params=params)
    summ["held_out_windows"] = "seeds 10^6..10^6+15 of the 640x480 street recipe, N=6"
    summ["training"] = (f"{int(meta.get('train', 0))} windows, {int(meta.get('steps', 0))} Adam steps on plain-GEM "
                        "outputs")
    return summ, prop


if __name__ == "__main__":
    main()
