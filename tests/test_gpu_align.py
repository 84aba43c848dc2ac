"""GPU parity of the keyframe alignments (sec. III-B) with the oracle: the rigid point-to-plane
alignment at the 640x480 keyframe size, and the 7-DoF alignment (motion and relative depth
scale, Levenberg-Marquardt).  Bars: pose 6-vector |d| <= 1e-5 (5e-4 on GEM outputs), scale
rel 1e-5, status equal, costs rel 1e-3, covariance 1e-2 of its norm (LM's accept / reject
decisions compare costs that the GPU sums from FP32 terms; near convergence a decision can go
the other way, which moves the state by no more than the converged step)."""
import numpy as np
import pytest
import torch

from oracle import align as oalign
from oracle import geometry as geo
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


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_rigid_alignment_at_keyframe_size(lib):
    """Two 640x480 pairs (1% inverse-depth noise, random confidence), 10 Gauss-Newton steps."""
    pr = synth.make_pairs(2, H=480, W=640, seed=3_000_501, noise_rel=0.01, conf="random")
    ap = pr["params"]
    rng = np.random.default_rng(5)
    pose0 = np.stack([geo.left_update(p, np.concatenate([rng.uniform(-0.01, 0.01, 3), rng.uniform(-0.02, 0.02, 3)]))
                      for p in pr["pose_gt"]])
    print("rigid alignment 640x480, 2 pairs", flush=True)
    pose_g = dev(pose0, torch.float64)
    cov, st, status = lib.align_p2p(ap, dev(pr["idepth1"]), dev(pr["idepth2"]), dev(pr["conf2"]), pose_g)
    pose_o = pose0.copy()
    ocov, ost, ostatus = oalign.align_p2p(ap, pr["idepth1"], pr["idepth2"], pr["conf2"], pose_o)
    print("pose diff", np.abs(np_(pose_g) - pose_o).max(), "stats", np_(st), ost)
    assert np.array_equal(np_(status), ostatus)
    assert np.abs(np_(pose_g) - pose_o).max() <= 1e-5
    np.testing.assert_allclose(np_(st)[:, :2], ost[:, :2], rtol=1e-3)
    c = np_(cov).reshape(-1, 6, 6)
    for i in range(2):
        assert np.abs(c[i] - ocov[i].reshape(6, 6)).max() <= 1e-3 * np.abs(ocov[i]).max()


@pytest.mark.parametrize("H,W,n", [(96, 128, 3), (480, 640, 2)])
def test_sim3_alignment(lib, H, W, n):
    pr = synth.make_pairs(n, H=H, W=W, seed=3_000_611 + H, planar=(H < 200), noise_rel=0.0 if H < 200 else 0.01,
                          conf="ones" if H < 200 else "random")
    ap = dict(pr["params"], gn_steps=15)
    rng = np.random.default_rng(H)
    s_true = np.array([0.8, 1.25, 1.05])[:n]
    r1 = pr["idepth1"] * s_true[:, None, None].astype(np.float32)
    pose0 = np.stack([geo.left_update(p, np.concatenate([rng.uniform(-0.02, 0.02, 3), rng.uniform(-0.03, 0.03, 3)]))
                      for p in pr["pose_gt"]])
    s0 = np.ones(n)
    print(f"sim(3) alignment {W}x{H}, {n} pairs", flush=True)
    pose_g, s_g = dev(pose0, torch.float64), dev(s0, torch.float64)
    cov, st, status = lib.align_sim3(ap, dev(r1), dev(pr["idepth2"]), dev(pr["conf2"]), pose_g, s_g)
    pose_o, s_o = pose0.copy(), s0.copy()
    ocov, ost, ostatus = oalign.align_sim3(ap, r1.astype(np.float32), pr["idepth2"], pr["conf2"], pose_o, s_o)
    gp, gs, gst = np_(pose_g), np_(s_g), np_(st)
    print("scale gpu", gs, "oracle", s_o, "true", s_true)
    print("pose diff", np.abs(gp - pose_o).max(), "vs truth", np.abs(gp - pr["pose_gt"]).max())
    print("stats gpu", gst.tolist(), "oracle", ost.tolist())
    assert np.array_equal(np_(status), ostatus)
    assert np.abs(gp - pose_o).max() <= 1e-5
    np.testing.assert_allclose(gs, s_o, rtol=1e-5)
    np.testing.assert_allclose(gst[:, :2], ost[:, :2], rtol=1e-3)
    c = np_(cov).reshape(-1, 7, 7)
    for i in range(n):
        oc = ocov[i].reshape(7, 7)
        assert np.linalg.norm(c[i] - oc) <= 1e-2 * np.linalg.norm(oc)
    # 1% inverse-depth noise and random confidence at 640x480 leave a scale error of a few 1e-3
    assert np.abs(gs / s_true - 1).max() < (2e-3 if H < 200 else 5e-3)


def test_sim3_single_plane_is_singular(lib):
    H, W = 30, 40
    ap = dict(H=H, W=W, fx=40.0, fy=40.0, cx=20.0, cy=15.0, robust=0, robust_scale=0.02, gn_steps=3,
              normal_disc_rel=0.05, scale_s=1.0)
    rho = dev(np.full((1, H, W), 0.5))
    pose = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    s = torch.ones(1, dtype=torch.float64, device="cuda")
    cov, st, status = lib.align_sim3(ap, rho, rho.clone(), torch.ones_like(rho), pose, s)
    from paper_2104_06800_amd.binding import ESINGULAR
    assert int(np_(status)[0]) == ESINGULAR
    assert np.array_equal(np_(pose), np.zeros((1, 6))) and np_(s)[0] == 1.0
    assert np.isnan(np_(cov)).all()


def test_alignment_of_gem_outputs(lib):
    """The keyframe workload: two 640x480, N=8 windows of one room (with depth priors) per
    pair, GEM on each, then window b's inverse depth and confidence aligned to window a's,
    starting from the chained visual-odometry estimate (the true relative pose moved by up to
    1 deg and 3 cm) with the Cauchy kernel; the discontinuity test of the normals is widened
    to 20% for maps that carry the prior's 5% noise.  GPU against the oracle on the same GEM
    outputs: pose to 5e-4 (FP32 terms; two orders below the estimate's own error), initial
    cost rel 1e-4, final cost and count at the GPU's final pose.  Against the truth the
    estimate stays within twice the start's error bound: map 1's per-pixel noise makes its
    central-difference normals noise (the depth step between neighbours is ~0.2% of depth),
    so these maps do not pin the pose better than the start; with exact normals the same
    start converges to a few 1e-3 (the synthetic pair tests)."""
    ap = None
    maps1, maps2, confs, truth, gt1 = [], [], [], [], []
    for k in range(2):
        wa, wb, pose_ba = synth.keyframe_pair(k)
        outs = []
        for w in (wa, wb):
            p = w["params"]
            b = lib.alloc(p, w["flow"], w["pose_init"], w["prior_idepth"], w["prior_pose"])
            lib.run(p, b, iters=p["iters"])
            outs.append((np_(b["idepth"]).copy(), np_(b["conf"]).copy()))
        maps1.append(outs[0][0])
        gt1.append(wa["idepth_gt"])
        maps2.append(outs[1][0])
        confs.append(outs[1][1])
        truth.append(pose_ba)
        if ap is None:
            fx, fy, cx, cy = wa["intr"]
            ap = dict(H=wa["params"]["H"], W=wa["params"]["W"], fx=fx, fy=fy, cx=cx, cy=cy, robust=1,
                      robust_scale=0.02, gn_steps=10, normal_disc_rel=0.2, scale_s=1.0)
    r1, r2, c2 = np.stack(maps1), np.stack(maps2), np.stack(confs)
    for k in range(2):
        e = np.median(np.abs(r1[k] - gt1[k]) / gt1[k])
        print(f"pair {k}: GEM median inverse-depth rel error {e:.4f}")
        assert e < 0.06                 # the start from the 5%-noise prior holds
    print("alignment of GEM outputs: 2 pairs 640x480", flush=True)
    rng = np.random.default_rng(17)
    pose0 = np.stack([geo.left_update(p, np.concatenate([np.deg2rad(rng.uniform(-1, 1, 3)), rng.uniform(-0.03, 0.03, 3)]))
                      for p in truth])
    pose_g = dev(pose0, torch.float64)
    cov, st, status = lib.align_p2p(ap, dev(r1), dev(r2), dev(c2), pose_g)
    pose_o = pose0.copy()
    ocov, ost, ostatus = oalign.align_p2p(ap, r1, r2, c2, pose_o)
    gp = np_(pose_g)
    err = np.abs(gp - np.stack(truth)).max(1)
    print("pose diff to oracle", np.abs(gp - pose_o).max(), "error vs truth", err, "stats", np_(st).tolist())
    assert np.array_equal(np_(status), ostatus)
    # per-pixel terms in FP32 on maps with 4% depth noise: the GPU and the oracle agree to
    # 5e-4, two orders below the estimate's own error against the truth
    assert np.abs(gp - pose_o).max() <= 5e-4
    gst = np_(st)
    np.testing.assert_allclose(gst[:, 0], ost[:, 0], rtol=1e-4)
    # the final cost is checked at the GPU's own final pose (nearest-pixel association makes
    # the cost jump between poses 1e-4 apart)
    for i in range(2):
        nrm, nv = oalign.normals(r1[i], ap["fx"], ap["fy"], ap["cx"], ap["cy"], ap["normal_disc_rel"])
        _, _, c_at, n_at = oalign.linearize(ap, r1[i], nrm, nv, r2[i], c2[i], gp[i])
        assert gst[i, 1] == pytest.approx(c_at, rel=1e-4) and abs(gst[i, 2] - n_at) <= max(2, 1e-4 * n_at)
    assert (err < 0.06).all()
