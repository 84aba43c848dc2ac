"""GPU: the whole-window entry points and the launch timers.

voldor_run and voldor_batch_run promise the results of the equivalent sequence of
per-step calls bit for bit (same kernels, same launch order, the flow layout built once
instead of per call), so these tests compare with exact equality.  Their parity with the
oracle follows from the per-step parity tests.
"""
import numpy as np
import pytest
import torch

from paper_2104_06800_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("idepth", "rigid", "pose", "conf", "stats", "idepth_coarse", "rigid_coarse")


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06800_amd.binding import Voldor
    v = Voldor(0)
    yield v
    v.close()


def alloc(lib, w):
    p = w["params"]
    return lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"),
                     w.get("prior_weight"))


def host(b):
    torch.cuda.synchronize()
    return {k: b[k].detach().cpu().numpy().copy() for k in KEYS}


def assert_same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def windows():
    out = [synth.make_window(1, 0), synth.make_window(3, 1, H=53, W=70, N=4),
           synth.make_window(1, 2, H=40, W=61, N=5)]
    out[2]["params"]["tile"] = 16
    return out


def test_run_equals_step_sequence(lib):
    w = synth.make_window(1, 3)
    p = w["params"]
    a, b = alloc(lib, w), alloc(lib, w)
    I = p["iters"]
    print(f"run vs steps: {p['W']}x{p['H']} N={p['N']} iters={I}", flush=True)
    lib.run(p, a, iters=I)
    lib.init_idepth(p, b)
    for it in range(I):
        lib.gem_step(p, b, it)
    lib.finalize(p, b, I - 1)
    assert_same(host(a), host(b))


def test_run_without_init_continues_from_given_depth(lib):
    w = synth.make_window(1, 4)
    p = w["params"]
    a, b = alloc(lib, w), alloc(lib, w)
    for t in (a, b):
        t["idepth"].copy_(torch.as_tensor(w["idepth_gt"], dtype=torch.float32).cuda())
    lib.run(p, a, iters=2, init=False)
    for it in range(2):
        lib.gem_step(p, b, it)
    lib.finalize(p, b, 1)
    assert_same(host(a), host(b))


def test_warm_start_equals_step_sequence(lib):
    w = synth.make_window(1, 5)
    p = w["params"]
    a, b = alloc(lib, w), alloc(lib, w)
    for t in (a, b):
        t["idepth"].copy_(torch.as_tensor(w["idepth_gt"] * 1.1, dtype=torch.float32).cuda())
    lib.run(p, a, iters=2, init=False, first_iter=3)
    for it in (3, 4):
        lib.gem_step(p, b, it)
    lib.finalize(p, b, 4)
    assert_same(host(a), host(b))


def test_batch_run_equals_individual_runs(lib):
    ws = windows()
    iters = 3
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    single = [(w["params"], alloc(lib, w)) for w in ws]
    print("batch of", [(p["W"], p["H"], p["N"], p.get("P", 0)) for p, _ in batch], flush=True)
    lib.batch_run(batch, iters)
    for p, b in single:
        lib.run(p, b, iters=iters)
    for (_, x), (_, y) in zip(batch, single):
        hx = host(x)
        assert_same(hx, host(y))
        assert np.isfinite(hx["stats"]).all()


def test_batched_windows_meet_the_oracle(lib):
    """Each window of a batch (64x48 N=3; 70x53 N=4 with a depth prior; 61x40 N=5 on 16x16
    tiles) against the oracle's plain GEM run independently from the same seed: 5
    iterations from the Philox initial depth, then the final E-step and statistics."""
    from oracle import gem as ogem
    ws = windows()
    iters = 5
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    print("batch vs oracle:", [(p["W"], p["H"], p["N"], p.get("P", 0)) for p, _ in batch], flush=True)
    lib.batch_run(batch, iters)
    for w, (p, b) in zip(ws, batch):
        g = host(b)
        ob = ogem.alloc_buffers(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))
        ost = ogem.run(p, ob, iters=iters)
        rho_frac = np.mean(np.abs(g["idepth"] - ob["idepth"]) <= 1e-3 * ob["idepth"])
        q_frac = np.mean(np.abs(g["rigid"] - ob["rigid"]) <= 1e-3)
        dpose = np.abs(g["pose"] - ob["pose"]).max()
        print(f"{p['W']}x{p['H']} N={p['N']} P={p.get('P', 0)}: rho {rho_frac:.4f} q {q_frac:.4f} "
              f"pose {dpose:.2e} loglik {g['stats'][0]:.9g} / {ost[0]:.9g} energy {g['stats'][1]:.9g} / "
              f"{ost[1]:.9g}", flush=True)
        assert rho_frac >= 0.99 and q_frac >= 0.99
        assert dpose <= 1e-4
        assert g["stats"][0] == pytest.approx(ost[0], rel=1e-3)
        assert g["stats"][1] == pytest.approx(ost[1], rel=1e-3)


def test_batch_graph_replay_and_direct_launches_agree(lib):
    """The captured graph, its replay on a later identical call and the uncaptured batched
    launches all give the individual runs' results."""
    ws = windows()
    ws.append(synth.make_window(1, 9, H=30, W=44, N=2))
    ws[-1]["params"].update(pose_gn_steps=0, n_candidates=9)
    iters = 2
    single = [(w["params"], alloc(lib, w)) for w in ws]
    for p, b in single:
        lib.run(p, b, iters=iters)
    ref = [host(b) for _, b in single]
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    pose0 = [b["pose"].clone() for _, b in batch]
    for graph, rep in ((True, 0), (True, 1), (False, 0)):
        for (p, b), p0 in zip(batch, pose0):
            b["pose"].copy_(p0)
        lib.batch_run(batch, iters, graph=graph)
        for (_, b), r in zip(batch, ref):
            assert_same(host(b), r)


def test_batch_run_with_uneven_pose_steps_equals_individual_runs(lib):
    """Windows with 0, 1 and 3 Gauss-Newton steps per frame (different step counts N*G):
    the batched pose passes and per-step solves cover only the windows that have step s."""
    ws = [synth.make_window(1, 20), synth.make_window(1, 21, H=40, W=52, N=5),
          synth.make_window(3, 22, H=36, W=48, N=4)]
    for w, G in zip(ws, (1, 3, 0)):
        w["params"]["pose_gn_steps"] = G
    iters = 2
    single = [(w["params"], alloc(lib, w)) for w in ws]
    for p, b in single:
        lib.run(p, b, iters=iters)
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    print("pose steps per window", [p["N"] * p["pose_gn_steps"] for p, _ in batch], flush=True)
    lib.batch_run(batch, iters)
    for (_, x), (_, y) in zip(batch, single):
        assert_same(host(x), host(y))


def test_batch_run_rejects_bad_arguments(lib):
    from paper_2104_06800_amd.binding import VoldorError
    ws = windows()[:2]
    batch = [(w["params"], alloc(lib, w)) for w in ws]
    with pytest.raises(VoldorError):
        lib.batch_run(batch, 0)
    with pytest.raises(VoldorError):
        lib.batch_run([], 1)
    bad = dict(ws[1]["params"])
    bad["n_candidates"] = 2
    with pytest.raises(VoldorError):
        lib.batch_run([batch[0], (bad, batch[1][1])], 1)


def test_timers_count_bracketed_launches(lib):
    from paper_2104_06800_amd.binding import TIMER_COARSE, TIMER_LOCAL, TIMER_POSE
    w = synth.make_window(1, 0)
    p = w["params"]
    b = alloc(lib, w)
    lib.timing(True)
    lib.run(p, b, iters=3)
    lib.level_step(p, b, 1, 1)
    got = {t: lib.timing_read(t) for t in (TIMER_LOCAL, TIMER_COARSE, TIMER_POSE)}
    lib.timing(False)
    # local: 3 fused passes + the level_step; the final E-step alone is not bracketed
    assert got[TIMER_LOCAL][1] == 4 and got[TIMER_COARSE][1] == 3 and got[TIMER_POSE][1] == 3
    assert all(ms > 0 for ms, _ in got.values())
    assert lib.timing_read(TIMER_LOCAL) == (0.0, 0)
    lib.run(p, b, iters=1)
    assert lib.timing_read(TIMER_LOCAL) == (0.0, 0)
    # one class enabled: only its launches are bracketed
    lib.timing(True, timers=(TIMER_POSE,))
    lib.run(p, b, iters=2)
    assert lib.timing_read(TIMER_POSE)[1] == 2
    assert lib.timing_read(TIMER_LOCAL) == (0.0, 0) and lib.timing_read(TIMER_COARSE) == (0.0, 0)
    lib.timing(False)


def test_timing_rejects_bad_mask(lib):
    from paper_2104_06800_amd import binding
    assert binding._LIB.voldor_timing(lib._h, 8) == binding.EINVAL
    assert binding._LIB.voldor_timing(lib._h, -1) == binding.EINVAL
