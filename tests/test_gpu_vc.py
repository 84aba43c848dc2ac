"""GPU parity of the visibility-coverage scores (sec. III-A "VO Stride and Keyframe
Selection") with the oracle: the counts, the three scores and the first pose below the
threshold must agree exactly (both sides take every inside / cell decision in FP64)."""
import numpy as np
import pytest
import torch

from oracle import vc as ovc
from paper_2104_06800_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06800_amd.binding import Voldor
    v = Voldor(0)
    yield v
    v.close()


def dev(a, dt=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def check(lib, vp, rho, conf, poses, tau):
    print(f"vc: {vp['W']}x{vp['H']} cell {vp['cell']} poses {len(poses)} conf {conf is not None}", flush=True)
    out, first = lib.vc_scores(vp, dev(rho), None if conf is None else dev(conf), poses, tau)
    torch.cuda.synchronize()
    ref, rfirst = ovc.vc_scores(vp, rho.astype(np.float32), None if conf is None else conf.astype(np.float32),
                                poses, tau)
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), (got[:4], ref[:4])
    assert int(first.cpu()[0]) == rfirst
    return got


def street_case(H=None, W=None):
    w = synth.make_window(2, 3, noise=False, H=H, W=W)
    p = w["params"]
    vp = dict(H=p["H"], W=p["W"], fx=p["fx"], fy=p["fy"], cx=p["cx"], cy=p["cy"], cell=8, conf_min=0.5)
    return w, vp


def test_street_window_against_its_frames(lib):
    """Ground-truth inverse depth of a driving window against its own frames' poses and a
    keyframe pose farther back, with a random confidence map."""
    w, vp = street_case()
    rng = np.random.default_rng(4)
    conf = rng.uniform(0, 1, w["idepth_gt"].shape)
    poses = np.concatenate([w["pose_gt"], [[0.0, 0.05, 0.0, 0.3, 0.0, -9.0]]])
    got = check(lib, vp, w["idepth_gt"], conf, poses, 0.7)
    print('VC per frame:', np.round(got[:, 2], 4))
    check(lib, dict(vp, cell=1), w["idepth_gt"], None, poses, 0.9)


def test_random_depth_holes_and_poses(lib):
    rng = np.random.default_rng(5)
    H, W = 97, 131
    vp = dict(H=H, W=W, fx=90.0, fy=88.0, cx=64.3, cy=47.8, cell=4, conf_min=0.25)
    rho = rng.uniform(0.05, 1.0, (H, W))
    rho[rng.uniform(size=(H, W)) < 0.1] = np.nan
    rho[rng.uniform(size=(H, W)) < 0.02] = -0.5
    conf = rng.uniform(0, 1, (H, W))
    conf[0, :5] = np.nan
    poses = np.concatenate([rng.normal(0, [0.05] * 3 + [0.5] * 3, (60, 6)),
                            [[0, 0, 0, 0, 0, -30.0], [0, 0, 0, 0, 0, 0]]])
    check(lib, vp, rho, conf, poses, 0.5)
    check(lib, dict(vp, cell=7), rho, None, poses, 0.95)


@pytest.mark.parametrize("H,W,cell", [(1, 1, 1), (2, 3, 8), (5, 1, 2), (64, 64, 1024), (33, 65, 32)])
def test_edge_shapes(lib, H, W, cell):
    rng = np.random.default_rng(H * 1000 + W)
    vp = dict(H=H, W=W, fx=20.0, fy=20.0, cx=W / 2 - 0.3, cy=H / 2 + 0.2, cell=cell, conf_min=0.0)
    rho = rng.uniform(0.2, 1.0, (H, W))
    poses = rng.normal(0, [0.02] * 3 + [0.2] * 3, (5, 6))
    check(lib, vp, rho, None, poses, 0.5)


def test_no_depth_pixels_and_many_poses(lib):
    H, W = 40, 56
    vp = dict(H=H, W=W, fx=40.0, fy=40.0, cx=27.7, cy=19.6, cell=4, conf_min=0.0)
    got = check(lib, vp, np.full((H, W), np.nan), None, np.zeros((3, 6)), 0.5)
    assert (got == 0).all()
    rng = np.random.default_rng(6)
    poses = rng.normal(0, [0.01] * 3 + [0.1] * 3, (1024, 6))
    check(lib, vp, rng.uniform(0.1, 1.0, (H, W)), None, poses, 0.3)


def test_bad_arguments_rejected(lib):
    from paper_2104_06800_amd.binding import VoldorError
    vp = dict(H=8, W=8, fx=10.0, fy=10.0, cx=4.0, cy=4.0, cell=2, conf_min=0.0)
    rho = dev(np.ones((8, 8)))
    for bad in (dict(cell=0), dict(fx=0.0), dict(H=0)):
        with pytest.raises(VoldorError):
            lib.vc_scores(dict(vp, **bad), rho if "H" not in bad else dev(np.ones((0, 8))), None,
                          np.zeros((1, 6)), 0.5)
    with pytest.raises(VoldorError):
        lib.vc_scores(vp, rho, None, np.zeros((1025, 6)), 0.5)
