"""Pins of the oracle's building blocks against things other than itself: published
known answers, SciPy distributions and rotations, quadrature, finite differences,
closed forms and the independent ray-casting generator."""
import os

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.spatial.transform import Rotation

from oracle import fisk, geometry as geo, philox
from oracle import gem
from paper_2104_06800_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_philox_uniforms_are_uniform_and_exact():
    u = philox.uniforms(np.arange(1 << 18), 0, 3, 1, philox.PURPOSE_CAND, 7, 12345)
    assert u.shape == (1 << 18, 4)
    assert (u >= 0).all() and (u < 1).all()
    # exact 24-bit grid: u * 2^24 is an integer
    assert np.array_equal(u * 2.0 ** 24, np.floor(u * 2.0 ** 24))
    for k in range(4):
        counts, _ = np.histogram(u[:, k], bins=64, range=(0, 1))
        chi2 = stats.chisquare(counts).pvalue
        assert chi2 > 1e-4
    # words are decorrelated and counters / purposes give different streams
    assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < 0.01
    v = philox.uniforms(np.arange(1 << 10), 0, 3, 1, philox.PURPOSE_INIT, 7, 12345)
    assert not np.array_equal(u[:1 << 10], v)


# ----------------------------------------------------------------------------- Fisk
@pytest.mark.parametrize("alpha,beta", [(0.5, 2.0), (0.8, 2.0), (0.7, 1.5), (1.1, 3.0)])
def test_fisk_pdf_matches_scipy(alpha, beta):
    r = np.linspace(0.01, 10, 500)
    np.testing.assert_allclose(fisk.fisk_pdf(r, alpha, beta), stats.fisk.pdf(r, c=beta, scale=alpha),
                               rtol=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.5, 2.0), (0.8, 2.0), (0.7, 1.5), (1.1, 3.0)])
def test_planar_density_normalised(alpha, beta):
    val, _ = integrate.quad(lambda r: 2 * np.pi * r * fisk.planar_density(r, alpha, beta), 0, np.inf,
                            limit=400)
    assert abs(val - 1.0) < 1e-7


def test_planar_density_beta2_closed_form():
    a = 0.5
    assert fisk.planar_density(0.0, a, 2.0) == pytest.approx(1 / (np.pi * a * a), rel=1e-14)
    r = np.linspace(0, 6, 50)
    np.testing.assert_allclose(fisk.planar_density(r, a, 2.0),
                               1 / (np.pi * a * a * (1 + r * r / (a * a)) ** 2), rtol=1e-13)
    # MIE cost for shape 2 collapses to log1p(c s^2), c = pi a^2 L0, s = 1 + r^2/a^2
    L0 = 1 / (np.pi * 64)
    c = np.pi * a * a * L0
    np.testing.assert_allclose(fisk.flow_term(r * r, a, 2.0, L0), np.log1p(c * (1 + r * r / (a * a)) ** 2),
                               rtol=1e-13)
    # inlier / outlier crossover near 1.94 px for a = 0.5, R = 8
    rc = a * np.sqrt(np.sqrt(1 / c) - 1)
    assert rc == pytest.approx(1.94, abs=0.01)
    assert fisk.flow_term(rc * rc, a, 2.0, L0) == pytest.approx(np.log(2.0), rel=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.5, 2.0), (0.8, 2.0), (0.7, 1.5), (1.1, 3.0)])
def test_flow_weight_is_derivative_of_cost(alpha, beta):
    L0 = 1 / (np.pi * 64)
    x = np.linspace(0.05, 30, 200)
    h = 1e-6 * x
    fd = (fisk.flow_term(x + h, alpha, beta, L0) - fisk.flow_term(x - h, alpha, beta, L0)) / (2 * h)
    np.testing.assert_allclose(fisk.flow_weight(x, alpha, beta, L0), fd, rtol=1e-6)


def test_prior_terms_match_gaussian_uniform_mixture():
    cs, cu = 0.05, 2.0
    lk = fisk.prior_log_kappa(cs, cu)
    rho_hat = np.array([0.1, 0.3, 0.9])
    rho = np.array([0.1, 0.33, 0.7])
    sig = cs * rho_hat
    N = stats.norm.pdf(rho_hat - rho, scale=sig)
    U = 1.0 / (cu * rho_hat)
    z = (rho_hat - rho) / sig
    np.testing.assert_allclose(fisk.prior_term(z, lk), np.log((N + U) / N), rtol=1e-12)
    pi = np.array([0.5, 0.8, 0.2])
    np.testing.assert_allclose(fisk.prior_posterior(z, lk, pi), pi * N / (pi * N + (1 - pi) * U), rtol=1e-12)
    assert fisk.prior_posterior(0.0, lk, 0.0) == 0.0


# ----------------------------------------------------------------------------- geometry
def test_rotations_match_scipy():
    rng = np.random.default_rng(0)
    for w in list(rng.normal(size=(20, 3)) * 0.7) + [np.zeros(3), np.array([1e-7, -2e-7, 3e-8]),
                                                   np.array([0, 0, np.pi - 1e-3]),
                                                   np.array([1.0, 2.0, 2.0]) / 3 * (np.pi - 1e-6)]:
        R = geo.exp_so3(w)
        np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=1e-13)
        w2 = geo.log_so3(R)
        np.testing.assert_allclose(Rotation.from_rotvec(w2).as_matrix(), R, atol=1e-10)


def test_left_update_composes():
    rng = np.random.default_rng(1)
    p = np.concatenate([rng.normal(size=3) * 0.2, rng.normal(size=3)])
    d = np.concatenate([rng.normal(size=3) * 0.01, rng.normal(size=3) * 0.01])
    q = geo.left_update(p, d)
    E = Rotation.from_rotvec(d[:3]).as_matrix()
    R = Rotation.from_rotvec(p[:3]).as_matrix()
    np.testing.assert_allclose(Rotation.from_rotvec(q[:3]).as_matrix(), E @ R, atol=1e-13)
    np.testing.assert_allclose(q[3:], E @ p[3:] + d[3:], atol=1e-13)


def test_bilinear_exact_on_affine_fields_and_edges():
    H, W = 7, 9
    V, U = np.mgrid[0:H, 0:W].astype(float)
    f = np.stack([0.3 * U - 1.7 * V + 2.0, -0.2 * U + 0.1 * V - 5.0], -1)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, W - 1, 300)
    y = rng.uniform(0, H - 1, 300)
    x[:3] = [W - 1, 0, W - 1]
    y[:3] = [H - 1, H - 1, 0]
    val, ok = geo.bilinear(f, x, y)
    assert ok.all()
    np.testing.assert_allclose(val[:, 0], 0.3 * x - 1.7 * y + 2.0, atol=1e-12)
    np.testing.assert_allclose(val[:, 1], -0.2 * x + 0.1 * y - 5.0, atol=1e-12)
    _, ok = geo.bilinear(f, np.array([-1e-9, W - 1 + 1e-9, 2.0]), np.array([1.0, 1.0, H - 1 + 1e-6]))
    assert not ok.any()
    g = f.copy()
    g[3, 4] = np.nan
    _, ok = geo.bilinear(g, np.array([3.5, 4.0, 5.5]), np.array([2.5, 3.0, 3.0]))
    assert list(ok) == [False, False, True]


def test_reprojection_matches_ray_cast_flows():
    """Independent pin: the generator ray-casts the scene and projects hits; the oracle
    reprojects x~/rho through the pose 6-vector.  At the true depth and pose the first
    frame's rigid flow equals the noise-free observed flow."""
    w = synth.make_window(1, 3, noise=False)
    win = w["params"]
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    ww = gem.Window(win, b)
    V, U = np.mgrid[0:win["H"], 0:win["W"]]
    rho = w["idepth_gt"]
    R, t = geo.pose_rt(w["pose_gt"][0])
    px, py, ok = geo.project(geo.scaled_point(R, t, ww.rays(U, V), rho), *ww.intr)
    assert ok.all()
    fl = w["flow"][0].astype(np.float64)
    np.testing.assert_allclose(px - U, fl[..., 0], atol=2e-5)   # flows are stored as float32
    np.testing.assert_allclose(py - V, fl[..., 1], atol=2e-5)
    r2, okr = ww.flow_residuals(U.ravel(), V.ravel(), rho.ravel())
    assert np.max(r2[0]) < 1e-9


def test_reprojection_special_cases():
    win = synth.default_params(20, 30, 1, (40.0, 40.0, 15.0, 10.0))
    V, U = np.mgrid[0:20, 0:30]
    xt = geo.rays(U, V, 40.0, 40.0, 15.0, 10.0)
    rho = np.full((20, 30), 0.25)
    px, py, _ = geo.project(geo.scaled_point(np.eye(3), np.zeros(3), xt, rho), 40.0, 40.0, 15.0, 10.0)
    np.testing.assert_allclose(px, U, atol=1e-12)
    np.testing.assert_allclose(py, V, atol=1e-12)
    # fronto-parallel plane, translation along x: constant flow f * tx * rho
    tx = 0.3
    px, py, _ = geo.project(geo.scaled_point(np.eye(3), np.array([tx, 0, 0]), xt, rho), 40.0, 40.0, 15.0, 10.0)
    np.testing.assert_allclose(px - U, 40.0 * tx * 0.25, atol=1e-12)
    np.testing.assert_allclose(py - V, 0.0, atol=1e-12)
    del win
