"""Learned depth / rigidness proposal: training data from plain GEM on seeded synthetic
windows, the training driver, and the comparison of learned-initialised GEM with plain GEM.

Host logic only: every forward, backward and optimiser step runs in the library's kernels
(voldor_proposal_forward / voldor_proposal_train_step), every GEM run in its GEM kernels.

Windows follow the street recipe at 640x480 with N = 6 (synth workload 4).  Training targets
are plain GEM's outputs after its full iterations (inverse depth, rigidness maps, confidence),
not the ground truth: the proposal learns to start GEM where GEM would end.  Accuracy is
the median over static pixels of |rho - rho_gt| / rho_gt after median scaling
(rho * median(rho_gt / rho)), as for monocular depth.
"""
import time
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np
import torch

from . import synth
from .binding import NET_PARAMS, Voldor

# (c_in, c_out) of c1..c6 as stored; the real input channels of c1 are 2N and the real
# output channels of c6 are 1 + N
LAYER_CHANNELS = [(16, 64), (64, 128), (128, 128), (128, 128), (128, 64), (64, 32)]
TRAIN_SEED0 = 0              # training windows: k = 0, 1, ...
TEST_SEED0 = 1_000_000       # held-out windows: k = 10^6, 10^6 + 1, ...
WORKLOAD = 4


def init_params(seed, n_frames):
    """He-normal initial weights on the real channels, zero biases, as the flat FP32 vector
    the library takes (per layer: w [Cout][3][3][Cin], then b [Cout])."""
    rng = np.random.default_rng(seed)
    parts = []
    for L, (ci, co) in enumerate(LAYER_CHANNELS):
        ri = 2 * n_frames if L == 0 else ci
        ro = 1 + n_frames if L == len(LAYER_CHANNELS) - 1 else co
        w = np.zeros((co, 3, 3, ci), dtype=np.float32)
        w[:ro, :, :, :ri] = rng.standard_normal((ro, 3, 3, ri)) * np.sqrt(2.0 / (9 * ri))
        parts += [w.ravel(), np.zeros(co, dtype=np.float32)]
    out = np.concatenate(parts)
    assert out.size == NET_PARAMS
    return out


def tnorm_of(pose_init):
    return float(np.linalg.norm(np.asarray(pose_init)[0, 3:]))


def _window(k):
    return synth.make_window(WORKLOAD, k)


def generate(ks, workers=16):
    """Synthetic windows for seeds ks, generated in worker processes (CPU only)."""
    if workers <= 1:
        return [_window(k) for k in ks]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_window, ks))


def median_rel_error(rho, gt, static):
    rho = np.asarray(rho, dtype=np.float64)
    ok = static & np.isfinite(rho) & (rho > 0)
    s = np.median(gt[ok] / rho[ok])
    return float(np.median(np.abs(rho[ok] * s - gt[ok]) / gt[ok]))


class Dataset:
    """Windows on the GPU with plain GEM's outputs as targets."""

    def __init__(self, lib, windows, conf_min=0.5):
        self.items = []
        for w in windows:
            p = w["params"]
            b = lib.alloc(p, w["flow"], w["pose_init"])
            lib.run(p, b, iters=p["iters"])
            torch.cuda.synchronize()
            self.items.append(dict(
                params=p, flow=b["flow"], tnorm=tnorm_of(w["pose_init"]),
                rho_t=b["idepth"].clone(), q_t=b["rigid"].clone(),
                mask=(b["conf"] >= conf_min).to(torch.uint8).contiguous(),
                err_gem=median_rel_error(b["idepth"].cpu().numpy(), w["idepth_gt"], ~w["dynamic"])))
            del b


def train(lib, data, steps, lr=1e-3, lr_final=1e-4, lam=0.1, seed=0, params=None, log=print, log_every=50):
    """Adam over the windows in a seeded random order; learning rate decays geometrically
    from lr to lr_final.  Returns (FP32 parameters, loss history [steps][3])."""
    n_frames = data.items[0]["params"]["N"]
    net = lib.net_alloc(init_params(seed, n_frames) if params is None else params, train=True)
    loss = torch.zeros(3, dtype=torch.float64, device="cuda")
    hist = torch.zeros((steps, 3), dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    order = []
    t0 = time.time()
    for s in range(steps):
        if not order:
            order = list(rng.permutation(len(data.items)))
        it = data.items[order.pop()]
        rate = lr * (lr_final / lr) ** (s / max(1, steps - 1))
        lib.proposal_train_step(net, it["flow"], it["tnorm"], it["rho_t"], it["q_t"], it["mask"], lam, rate, s + 1,
                                loss)
        hist[s] = loss
        if log and ((s + 1) % log_every == 0 or s == steps - 1):
            h = hist[max(0, s + 1 - log_every):s + 1].mean(0).cpu().numpy()
            log(f"step {s + 1}/{steps}: loss {h[0]:.4f} (depth {h[1]:.4f}, rigidness {h[2]:.4f}), "
                f"{(time.time() - t0) / (s + 1) * 1e3:.1f} ms/step")
    torch.cuda.synchronize()
    return net["params"].cpu().numpy(), hist.cpu().numpy()


def save(path, params, meta):
    np.savez_compressed(path, params=np.asarray(params, dtype=np.float32),
                        **{k: np.asarray(v) for k, v in meta.items()})


def load(path):
    with np.load(path, allow_pickle=False) as z:
        params = z["params"].astype(np.float32)
        meta = {k: z[k] for k in z.files if k != "params"}
    if params.size != NET_PARAMS:
        raise ValueError(f"{path}: {params.size} parameters, expected {NET_PARAMS}")
    return params, meta


def learned_run(lib, net, p, b, iters, full_iters=None, fallback=None):
    """GEM from the proposal's start: the network's start of the window (library kernels,
    with the random start where its output is unusable), then iterations 0 .. iters-1 and the
    final E-step.  After a fallback the run continues to plain GEM's full schedule
    (full_iters, default the window's iteration count), which equals plain GEM's run bit for
    bit.  Returns True when the start fell back.  One device-to-host read (the flag)."""
    full = p["iters"] if full_iters is None else full_iters
    fb = torch.zeros(1, dtype=torch.int32, device=b["idepth"].device) if fallback is None else fallback
    lib.proposal_start(net, p, b, fb)
    lib.run(p, b, iters=iters, init=False)
    fell_back = bool(int(fb.cpu()[0]))
    if fell_back and iters < full:
        lib.run(p, b, iters=full - iters, init=False, first_iter=iters)
    return fell_back


def judged_run(lib, net, p, b, iters):
    """Plain GEM as the judge of the learned start: the learned start's run (learned_run with
    iters iterations) and plain GEM's full run on a copy of the window's buffers; the window
    keeps the one with the lower final MIE energy (a non-finite energy always loses).
    Returns "learned" or "plain"."""
    plain = {k: (v.clone() if torch.is_tensor(v) else v) for k, v in b.items()}
    learned_run(lib, net, p, b, iters)
    lib.run(p, plain, iters=p["iters"])
    e_l, e_p = (float(x["stats"][1].cpu()) for x in (b, plain))
    if np.isfinite(e_l) and (not np.isfinite(e_p) or e_l <= e_p):
        return "learned"
    for k, v in plain.items():
        if torch.is_tensor(v):
            b[k].copy_(v)
    return "plain"


def _timed(fn, reps=3):
    """Median wall time (ms) of fn() on the current stream, synchronised."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def compare(lib, net, windows, max_iters=None, reps=3, warm=True):
    """Plain GEM (random init, all iterations) against GEM started from the proposal, per
    window: the plain error and time, the learned-init error after each iteration count,
    and the time of the proposal plus the fewest iterations that reach the plain error.
    warm: the learned start runs the last k iterations of the schedule (iteration indices
    I-k .. I-1, narrow perturbations) rather than the first k."""
    out = []
    for w in windows:
        p = w["params"]
        I = p["iters"] if max_iters is None else max_iters
        static = ~w["dynamic"]
        b = lib.alloc(p, w["flow"], w["pose_init"])
        pose0 = b["pose"].clone()

        def plain():
            b["pose"].copy_(pose0)
            lib.run(p, b, iters=p["iters"])

        t_plain = _timed(plain, reps)
        e_plain = median_rel_error(b["idepth"].cpu().numpy(), w["idepth_gt"], static)
        tn = tnorm_of(w["pose_init"])

        def learned(k):
            # the network's start (written into the window's buffers by the library), then k
            # iterations; warm: the last k of the schedule (narrow perturbations)
            b["pose"].copy_(pose0)
            lib.proposal_start(net, p, b)
            lib.run(p, b, iters=k, init=False, first_iter=p["iters"] - k if warm else 0)

        t_net = _timed(lambda: lib.proposal_start(net, p, b), reps)
        errs, times = [], []
        for k in range(1, I + 1):
            times.append(_timed(lambda: learned(k), reps))
            e = median_rel_error(b["idepth"].cpu().numpy(), w["idepth_gt"], static)
            errs.append(e)
        rho0, _, _ = lib.proposal_forward(net, b["flow"], tn, p["idepth_min"], p["idepth_max"])
        e_init = median_rel_error(rho0.cpu().numpy(), w["idepth_gt"], static)
        out.append(dict(err_plain=e_plain, ms_plain=t_plain, err_proposal=e_init, err_learned=errs,
                        ms_learned=times, ms_proposal=t_net))
        del b
    return out


def summarize(res):
    """Set-level comparison: plain GEM's median (over windows) error and time; the fewest
    learned-start iterations k whose median error reaches it and the median time of the
    proposal plus those k iterations; the learned start's error after all iterations."""
    e_plain = float(np.median([r["err_plain"] for r in res]))
    ms_plain = float(np.median([r["ms_plain"] for r in res]))
    n = len(res[0]["err_learned"])
    e_k = [float(np.median([r["err_learned"][k] for r in res])) for k in range(n)]
    k_hit = next((k + 1 for k in range(n) if e_k[k] <= e_plain), None)
    ms_hit = None if k_hit is None else float(np.median([r["ms_learned"][k_hit - 1] for r in res]))
    return dict(windows=len(res), err_plain=e_plain, ms_plain=ms_plain, err_proposal=float(
        np.median([r["err_proposal"] for r in res])), err_learned_by_iters=e_k, iters_to_plain=k_hit,
        ms_to_plain_error=ms_hit, err_learned_full=e_k[-1], ms_proposal=float(np.median([r["ms_proposal"] for r in res])))
