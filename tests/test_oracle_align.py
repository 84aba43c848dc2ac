"""Pins of the oracle's point-to-plane inverse-depth alignment: exact fixed point on
piecewise-planar scenes, the fronto-parallel reduction to the inverse-depth difference,
finite-difference Jacobians, analytic plane normals, convergence and rank deficiency."""
import numpy as np
import pytest

from oracle import align, geometry as geo
from paper_2104_06800_amd import synth


@pytest.fixture(scope="module")
def pairs():
    return synth.make_pairs(3, H=120, W=160, planar=True, seed=3_000_017)


def _ap(p, **kw):
    return dict(p["params"], **kw)


def test_normals_match_analytic_plane():
    H, W = 40, 60
    fx = fy = 50.0
    cx, cy = W / 2, H / 2
    n_true = np.array([0.3, -0.2, -1.0])
    n_true /= np.linalg.norm(n_true)
    d = -3.0                                        # plane n . X = d, in front of the camera
    V, U = np.mgrid[0:H, 0:W]
    x = geo.rays(U, V, fx, fy, cx, cy)
    rho = (x @ n_true) / d                          # 1/z for X = z x on the plane
    n, ok = align.normals(rho, fx, fy, cx, cy, 0.05)
    assert ok[1:-1, 1:-1].all() and not ok[0].any() and not ok[:, -1].any()
    np.testing.assert_allclose(n[ok], np.broadcast_to(n_true, n[ok].shape), atol=1e-12)


def test_fronto_parallel_reduces_to_inverse_depth_difference():
    """On a fronto-parallel plane the point-to-plane residual equals Eq. 9's difference of
    inverse depths, rho1(l) - 1/Q_z (s = 1)."""
    H, W = 30, 40
    ap = dict(H=H, W=W, fx=40.0, fy=40.0, cx=20.0, cy=15.0, robust=0, robust_scale=0.02, gn_steps=1,
              normal_disc_rel=0.05, scale_s=1.0)
    rho1 = np.full((H, W), 0.5)
    rho2 = np.full((H, W), 0.4)
    nrm, nv = align.normals(rho1, 40.0, 40.0, 20.0, 15.0, 0.05)
    pose = np.array([0.0, 0.0, 0.0, 0.01, -0.02, 0.3])
    _, _, _, cnt, r, _, ok = align.linearize(ap, rho1, nrm, nv, rho2, np.ones((H, W)), pose, terms=True)
    assert cnt > 0
    Qz = 1.0 / 0.4 + 0.3
    np.testing.assert_allclose(r[ok], 0.5 - 1.0 / Qz, atol=1e-13)


def test_residual_vanishes_at_true_pose_on_planar_interior(pairs):
    """At the true pose every map-2 pixel whose associated map-1 pixel has a 3x3
    neighbourhood on one planar surface has a zero residual (float32 map storage aside),
    so the true pose is a fixed point up to the pixels that straddle creases and edges."""
    ap = _ap(pairs)
    for i in range(3):
        r1 = pairs["idepth1"][i]
        nrm = align.normals(r1, ap["fx"], ap["fy"], ap["cx"], ap["cy"], ap["normal_disc_rel"])
        _, g, _, cnt, r, _, ok = align.linearize(ap, r1, *nrm, pairs["idepth2"][i], pairs["conf2"][i],
                                                 pairs["pose_gt"][i], terms=True)
        assert cnt > 1000
        # recompute each pixel's association to find its 3x3 neighbourhood in map 1
        H, W = r1.shape
        V, U = np.mgrid[0:H, 0:W]
        R, t = geo.pose_rt(pairs["pose_gt"][i])
        X2 = geo.rays(U, V, ap["fx"], ap["fy"], ap["cx"], ap["cy"]) / pairs["idepth2"][i][..., None]
        Q = X2 @ R.T + t
        lx = np.clip(np.floor(ap["fx"] * Q[..., 0] / Q[..., 2] + ap["cx"] + 0.5), 1, W - 2).astype(int)
        ly = np.clip(np.floor(ap["fy"] * Q[..., 1] / Q[..., 2] + ap["cy"] + 0.5), 1, H - 2).astype(int)
        obj = pairs["object1"][i]
        same = np.ones((H, W), dtype=bool)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                same &= obj[ly + dy, lx + dx] == obj[ly, lx]
        sel = ok & same & (pairs["object2"][i] == obj[ly, lx])     # not occluded in camera 1
        assert sel.sum() > 0.8 * ok.sum()
        assert np.abs(r[sel]).max() < 1e-6


def test_jacobian_by_finite_differences(pairs):
    ap = _ap(pairs, robust_scale=1e6)               # Huber in its quadratic branch: cost = sum C r^2/2
    i = 0
    nrm = align.normals(pairs["idepth1"][i], ap["fx"], ap["fy"], ap["cx"], ap["cy"], ap["normal_disc_rel"])
    p0 = geo.left_update(pairs["pose_gt"][i], np.array([0.002, -0.001, 0.001, 0.01, 0.005, -0.01]))
    _, _, _, _, r0, J, ok = align.linearize(ap, pairs["idepth1"][i], *nrm, pairs["idepth2"][i],
                                            pairs["conf2"][i], p0, terms=True)
    for k in range(6):
        d = np.zeros(6)
        d[k] = 1e-7
        _, _, _, _, rp, _, okp = align.linearize(ap, pairs["idepth1"][i], *nrm, pairs["idepth2"][i],
                                                 pairs["conf2"][i], geo.left_update(p0, d), terms=True)
        _, _, _, _, rm, _, okm = align.linearize(ap, pairs["idepth1"][i], *nrm, pairs["idepth2"][i],
                                                 pairs["conf2"][i], geo.left_update(p0, -d), terms=True)
        same = ok & okp & okm
        fd = (rp - rm)[same] / 2e-7
        # the association is fixed within a step, so compare where it did not change
        good = np.abs(fd - J[same][:, k]) <= 1e-5 * (1 + np.abs(fd))
        assert good.mean() > 0.99


def test_converges_from_perturbation(pairs):
    ap = _ap(pairs)
    rng = np.random.default_rng(21)
    for i in range(3):
        dw = np.deg2rad(rng.uniform(-2, 2, 3))
        dt = rng.uniform(-0.05, 0.05, 3)
        p0 = geo.left_update(pairs["pose_gt"][i], np.concatenate([dw, dt]))
        p, cov, st, status = align.align_pair(ap, pairs["idepth1"][i], pairs["idepth2"][i],
                                              pairs["conf2"][i], p0)
        assert status == 0
        # converges to the true pose up to the pull of pixels associated across creases
        assert np.abs(p - pairs["pose_gt"][i]).max() < 1e-3
        assert st[1] < st[0]
        assert np.all(np.linalg.eigvalsh(cov.reshape(6, 6)) > 0)


def test_single_plane_is_singular():
    H, W = 30, 40
    ap = dict(H=H, W=W, fx=40.0, fy=40.0, cx=20.0, cy=15.0, robust=0, robust_scale=0.02, gn_steps=3,
              normal_disc_rel=0.05, scale_s=1.0)
    rho = np.full((1, H, W), 0.5)
    pose = np.zeros((1, 6))
    cov, st, status = align.align_p2p(ap, rho, rho.copy(), np.ones((1, H, W)), pose)
    assert status[0] == align.ESINGULAR
    assert np.array_equal(pose, np.zeros((1, 6)))


def test_cauchy_kernel_weights():
    r = np.linspace(-0.1, 0.1, 20)            # avoids the Huber kink at |r| = 0.02
    psi, w = align.robust(r, align.CAUCHY, 0.02)
    h = 1e-7
    dpsi = (align.robust(r + h, align.CAUCHY, 0.02)[0] - align.robust(r - h, align.CAUCHY, 0.02)[0]) / (2 * h)
    nz = r != 0
    np.testing.assert_allclose(w[nz], dpsi[nz] / r[nz], rtol=1e-6)
    psi, w = align.robust(r, align.HUBER, 0.02)
    dpsi = (align.robust(r + h, align.HUBER, 0.02)[0] - align.robust(r - h, align.HUBER, 0.02)[0]) / (2 * h)
    np.testing.assert_allclose(w[nz], dpsi[nz] / r[nz], rtol=1e-6)
