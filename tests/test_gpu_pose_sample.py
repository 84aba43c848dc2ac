"""GPU parity of the sampled pose M-step (sec. III-A "Uncertainty-aware Pose Estimation")
with the oracle.  Both sides draw the same Philox triplets and work in FP64 from the same
FP32 inputs, so the draws, the void samples, the inlier sets and the step counts agree
exactly, and the poses (the meanshift modes) and covariances to FP64 rounding of the
different summation orders: poses |d| <= 1e-7 (the pose bar is 1e-5), covariances 1e-6 of
their norm."""
import numpy as np
import pytest
import torch

from oracle import gem as ogem
from oracle import pose_sample as ops
from paper_2104_06800_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06800_amd.binding import Voldor
    v = Voldor(0)
    yield v
    v.close()


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def compare(lib, p, b, it, prm):
    ob = ogem.alloc_buffers(p, np_(b["flow"]), np_(b["pose"]))
    for k in ("idepth", "rigid"):
        ob[k][...] = np_(b[k])
    print(f"pose sample: {p['W']}x{p['H']} N={p['N']} S={prm['samples']} tries={prm['tries']}", flush=True)
    cov, info = lib.pose_sample(p, b, it, prm)
    ocov, oinfo = ops.pose_sample_step(p, ob, it, prm)
    g_pose, g_cov, g_info = np_(b["pose"]), np_(cov), np_(info)
    print("info gpu", g_info.tolist(), "oracle", oinfo.tolist())
    print(f"max |d pose| {np.abs(g_pose - ob['pose']).max():.2e}")
    np.testing.assert_array_equal(g_info, oinfo)
    assert np.abs(g_pose - ob["pose"]).max() <= 1e-7
    for t in range(p["N"]):
        assert np.linalg.norm(g_cov[t] - ocov[t]) <= 1e-6 * np.linalg.norm(ocov[t])
    return g_info


def exact(lib, N, k, perturbed):
    w = synth.make_window(1, k, noise=False, N=N)
    p = w["params"]
    b = lib.alloc(p, w["flow"], w["pose_init"] if perturbed else w["pose_gt"])
    b["idepth"].copy_(torch.as_tensor(w["idepth_gt"], dtype=torch.float32))
    b["rigid"].fill_(1.0)
    return w, p, b


def test_exact_window(lib):
    w, p, b = exact(lib, 2, 1, False)
    info = compare(lib, p, b, 0, dict(ops.DEFAULTS, samples=64))
    assert info[0, 0] == 64
    assert np.abs(np_(b["pose"])[0] - w["pose_gt"][0]).max() < 1e-5


def test_perturbed_poses(lib):
    w, p, b = exact(lib, 3, 2, True)
    compare(lib, p, b, 0, dict(ops.DEFAULTS, samples=128, tries=8))


@pytest.mark.parametrize("it", [1, 4])
def test_mid_run_state(lib, it):
    w = synth.make_window(1, 3)
    p = w["params"]
    b = lib.alloc(p, w["flow"], w["pose_init"])
    lib.init_idepth(p, b)
    for i in range(2):
        lib.gem_step(p, b, i)
    lib.rigidness_fb(p, b, it, 1)
    compare(lib, p, b, it, dict(ops.DEFAULTS, samples=256))


def test_full_size_street_window(lib):
    w = synth.make_window(2, 0)
    p = w["params"]
    b = lib.alloc(p, w["flow"], w["pose_init"])
    lib.init_idepth(p, b)
    for i in range(3):
        lib.gem_step(p, b, i)
    lib.rigidness_fb(p, b, 3, 1)
    compare(lib, p, b, 3, dict(ops.DEFAULTS, samples=256, tries=16))


def test_no_rigid_pixels_keep_the_pose(lib):
    w, p, b = exact(lib, 2, 4, True)
    b["rigid"].zero_()
    before = np_(b["pose"]).copy()
    cov, info = lib.pose_sample(p, b, 0, dict(ops.DEFAULTS, samples=32))
    assert np.array_equal(np_(b["pose"]), before)
    assert (np_(info) == 0).all()
    kinv = ops.kernel_inv_diag(before[0], ops.DEFAULTS)
    np.testing.assert_allclose(np_(cov)[0].reshape(6, 6), np.diag(1.0 / kinv), rtol=1e-12)


def test_bad_parameters_rejected(lib):
    from paper_2104_06800_amd.binding import VoldorError
    w, p, b = exact(lib, 2, 5, False)
    for bad in (dict(samples=0), dict(samples=4097), dict(tries=0), dict(sigma_w=0.0), dict(eps=-1.0)):
        with pytest.raises(VoldorError):
            lib.pose_sample(p, b, 0, dict(ops.DEFAULTS, **bad))
