"""GPU: the allocation-free whole-window entry point (voldor_run_noalloc).

It runs voldor_run's kernels on a static per-device scratch array instead of the
context's grown buffer, so its results must equal voldor_run's bit for bit.  Three calls in
a row, each on a smaller window than the one before (the array keeps the previous call's
contents), then a window too large for the array, which must be refused before anything
is enqueued.
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


def host(b):
    torch.cuda.synchronize()
    return {k: b[k].detach().cpu().numpy().copy() for k in KEYS}


def random_street(H, W, N, seed):
    """Flows of random content for a large window (the comparison is GPU against GPU)."""
    rng = np.random.default_rng(seed)
    f0 = 720.0 * W / 1216
    p = synth.default_params(H, W, N, (f0, f0, W / 2, H / 2), fisk_alpha=0.8, n_candidates=32,
                             idepth_min=0.005, idepth_max=0.5, seed=int(rng.integers(0, 2 ** 62)), iters=1)
    flow = rng.normal(0.0, 3.0, (N, H, W, 2)).astype(np.float32)
    flow[:, :, :8] = np.nan                       # a band of holes
    pose = np.zeros((N, 6))
    pose[:, 5] = -np.arange(1, N + 1) * 0.9
    pose[:, 1] = 0.01 * np.arange(1, N + 1)
    return dict(params=p, flow=flow, pose_init=pose)


def cases():
    big = random_street(352, 1216, 8, 7)            # the largest window the array holds
    mid = synth.make_window(3, 5, H=120, W=160, N=8)  # with a depth prior
    small = synth.make_window(1, 4)
    return [(big, 1), (mid, 3), (small, 5)]


def test_noalloc_run_equals_run_on_shrinking_windows(lib):
    for w, iters in cases():
        p = w["params"]
        print(f"noalloc vs run: {p['W']}x{p['H']} N={p['N']} P={p['P']} iters={iters}", flush=True)
        a = lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))
        b = lib.alloc(p, w["flow"], w["pose_init"], w.get("prior_idepth"), w.get("prior_pose"))
        lib.run(p, a, iters=iters)
        lib.run_noalloc(p, b, iters=iters)
        ha, hb = host(a), host(b)
        for k in KEYS:
            assert np.array_equal(ha[k], hb[k], equal_nan=True), k
        assert np.isfinite(hb["stats"]).all()


def test_noalloc_refuses_window_beyond_static_scratch(lib):
    from paper_2104_06800_amd.binding import VoldorError
    H, W, N = 1024, 2048, 8
    p = synth.default_params(H, W, N, (1000.0, 1000.0, W / 2, H / 2))
    b = lib.alloc(p, np.zeros((N, H, W, 2), np.float32), np.zeros((N, 6)))
    before = b["idepth"].clone()
    with pytest.raises(VoldorError, match="static area holds"):
        lib.run_noalloc(p, b, iters=1)
    torch.cuda.synchronize()
    assert torch.equal(b["idepth"], before)          # nothing was enqueued
