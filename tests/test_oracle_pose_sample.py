"""Pins of the oracle's sampled pose estimation (sec. III-A "Uncertainty-aware Pose
Estimation"): P3P against exact correspondences, the meanshift fixed point and symmetric
mixtures, the 3-sigma covariance fit against the truncated-Gaussian fixed point computed from
chi-square laws, the eigenvalue floor, q-proportional triplet draws, and the whole step on
an exact window."""
import numpy as np
import pytest
from scipy import optimize, stats
from scipy.spatial.transform import Rotation

from oracle import gem, geometry as geo, pose_sample as ps
from paper_2104_06800_amd import synth


def random_pose(rng, deg=20.0, tr=1.0):
    return np.concatenate([Rotation.random(random_state=rng).as_rotvec() * (deg / 180.0),
                           rng.normal(0, tr, 3)])


def test_p3p_recovers_the_true_pose_among_its_solutions():
    rng = np.random.default_rng(0)
    for _ in range(300):
        pose = random_pose(rng)
        R, t = geo.pose_rt(pose)
        X = rng.normal(0, 1, (3, 3)) + np.array([0, 0, 6.0])
        C = X @ R.T + t
        if (C[:, 2] <= 0.5).any():
            continue
        f = C / np.linalg.norm(C, axis=1, keepdims=True)
        sols = ps.p3p(X, f)
        assert 1 <= len(sols) <= 4
        err = min(np.abs(Rs - R).max() + np.abs(ts - t).max() for Rs, ts in sols)
        assert err < 1e-7
        for Rs, ts in sols:                      # every solution puts the points on their rays
            Cs = X @ Rs.T + ts
            assert (Cs[:, 2] > 0).all()
            np.testing.assert_allclose(Cs / np.linalg.norm(Cs, axis=1, keepdims=True), f, atol=1e-7)
            np.testing.assert_allclose(Rs @ Rs.T, np.eye(3), atol=1e-9)


def test_rigid_from_triads_inverts_a_motion():
    rng = np.random.default_rng(1)
    R, t = geo.pose_rt(random_pose(rng, 90))
    X = rng.normal(0, 1, (3, 3))
    Rs, ts = ps.rigid_from_triads(X, X @ R.T + t)
    np.testing.assert_allclose(Rs, R, atol=1e-12)
    np.testing.assert_allclose(ts, t, atol=1e-12)


def test_chart_is_the_inverse_of_the_left_update():
    rng = np.random.default_rng(2)
    for _ in range(50):
        m, d = random_pose(rng), np.concatenate([rng.normal(0, 0.2, 3), rng.normal(0, 0.5, 3)])
        p = geo.left_update(m, d)
        Rm, tm = geo.pose_rt(m)
        np.testing.assert_allclose(ps.chart(geo.pose_rt(p), Rm, tm), d, atol=1e-10)


def cluster(rng, center, kinv, n, scale=1.0):
    sd = 1.0 / np.sqrt(kinv)
    return np.array([geo.left_update(center, rng.normal(0, scale * sd)) for _ in range(n)])


def test_meanshift_stops_at_a_fixed_point_near_the_dense_mode():
    """The returned mode satisfies the meanshift condition (kernel-weighted mean of the
    samples' coordinates about it = 0) and lies at the dense cluster, not at the far one."""
    rng = np.random.default_rng(3)
    center = np.array([0.02, -0.01, 0.03, 0.1, 0.2, -1.5])
    kinv = ps.kernel_inv_diag(center, ps.DEFAULTS)
    far = geo.left_update(center, 8.0 / np.sqrt(kinv))
    samples = np.concatenate([cluster(rng, center, kinv, 120, 0.7), cluster(rng, far, kinv, 60, 0.7)])
    start = geo.left_update(center, 1.5 / np.sqrt(kinv))
    mode, steps = ps.meanshift(samples, start, kinv)
    Rm, tm = geo.pose_rt(mode)
    d = np.array([ps.chart(geo.pose_rt(s), Rm, tm) for s in samples])
    w = np.exp(-0.5 * (d * d * kinv).sum(1))
    assert np.sqrt(((w[:, None] * d).sum(0) / w.sum()) ** 2 @ kinv) < 1e-10
    Rc, tc = geo.pose_rt(center)
    assert np.sqrt((ps.chart((Rm, tm), Rc, tc) ** 2 * kinv).sum()) < 0.5
    assert steps < 100


def test_meanshift_of_a_symmetric_mixture_is_its_centre():
    """Samples in pairs exp(+d) M, exp(-d) M: by symmetry the mode is M exactly."""
    rng = np.random.default_rng(4)
    M = np.array([0.01, 0.02, -0.015, -0.3, 0.1, -1.0])
    kinv = ps.kernel_inv_diag(M, ps.DEFAULTS)
    ds = rng.normal(0, 0.6, (40, 6)) / np.sqrt(kinv)
    samples = np.array([geo.left_update(M, s * d) for d in ds for s in (1, -1)])
    mode, _ = ps.meanshift(samples, geo.left_update(M, 0.3 / np.sqrt(kinv)), kinv)
    np.testing.assert_allclose(mode, M, atol=1e-9)


def test_truncation_factor():
    """The share of a 6-D Gaussian's variance inside its 3-sigma region: E[x x^T | chi2_6 <= 9]
    = Sigma P(chi2_8 <= 9) / P(chi2_6 <= 9); checked against scipy and by quadrature of the
    radial law."""
    k = stats.chi2.cdf(9, 8) / stats.chi2.cdf(9, 6)
    assert ps.KAPPA == pytest.approx(k, rel=1e-13)
    from scipy import integrate
    num = integrate.quad(lambda r2: r2 / 6 * stats.chi2.pdf(r2, 6), 0, 9)[0]
    assert ps.KAPPA == pytest.approx(num / stats.chi2.cdf(9, 6), rel=1e-9)


def test_covariance_fit_of_a_gaussian_with_outliers_is_its_covariance():
    """20000 samples of a 6-D Gaussian plus 400 far outliers: the iterated 3-sigma fit (with
    the truncation factor) returns the Gaussian's covariance to sampling error, and the
    literal fit without the factor would shrink towards c = 0.43 of it (the fixed point of
    c = P(chi2_8 <= 9c) / P(chi2_6 <= 9c))."""
    c_lit = optimize.brentq(lambda c: stats.chi2.cdf(9 * c, 8) / stats.chi2.cdf(9 * c, 6) - c, 0.3, 0.49)
    assert 0.42 < c_lit < 0.44
    rng = np.random.default_rng(5)
    M = np.array([0.0, 0.01, 0.0, 0.2, -0.1, -1.2])
    A = rng.normal(0, 1, (6, 6))
    true = A @ A.T / 6 * 1e-5 + np.diag([1e-6] * 3 + [4e-5] * 3)
    L = np.linalg.cholesky(true)
    n = 20000
    d = rng.normal(0, 1, (n, 6)) @ L.T
    samples = np.array([geo.left_update(M, x) for x in d])
    out = np.array([geo.left_update(M, x) for x in rng.uniform(-1, 1, (400, 6)) * np.sqrt(np.diag(true)) * 40])
    kinv = 1.0 / np.diag(true) / 4
    Sig, n_in, rounds = ps.fit_covariance(np.concatenate([samples, out]), M, kinv, 1e-14)
    # sampling error of a covariance from ~n points: a few percent
    rel = np.linalg.norm(Sig - true) / np.linalg.norm(true)
    print(f"relative difference {rel:.3f}, inliers {n_in}, rounds {rounds}")
    assert rel < 0.05
    p_in = stats.chi2.cdf(9, 6)                 # a 6-D Gaussian's share inside 3 sigma
    assert abs(n_in - p_in * n) < 5 * np.sqrt(n * p_in * (1 - p_in))


def test_covariance_eigenvalues_are_floored():
    rng = np.random.default_rng(6)
    M = np.array([0.0, 0.0, 0.0, 0.0, 0.0, -1.0])
    d = np.zeros((200, 6))
    d[:, 3:5] = rng.normal(0, 1e-3, (200, 2))          # spread in a 2-D subspace only
    samples = np.array([geo.left_update(M, x) for x in d])
    kinv = ps.kernel_inv_diag(M, ps.DEFAULTS)
    Sig, _, _ = ps.fit_covariance(samples, M, kinv, 1e-9)
    lam = np.sort(np.linalg.eigvalsh(Sig))
    np.testing.assert_allclose(lam[:4], 1e-9, rtol=1e-6)
    assert lam[4] > 1e-7


def exact_window(N=2, k=1):
    w = synth.make_window(1, k, noise=False, N=N)
    win = dict(w["params"])
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    b["idepth"][...] = w["idepth_gt"]
    b["rigid"][...] = 1.0
    return w, win, b


def test_triplet_draws_follow_the_rigidness():
    """Pixels with q = 0 are never drawn; with q = 1/2 on the other half of the image an
    attempt is accepted with probability 1/4, so a point of 16 attempts finds a pixel with
    probability 1 - (3/4)^16."""
    w, win, b = exact_window()
    b["rigid"][...] = 0.5
    b["rigid"][0, :, :32] = 0.0
    trip = ps.draw_triplets(win, b, 1, 0, 2000, 16)
    drawn = trip[trip >= 0]
    assert (drawn % win["W"] >= 32).all()
    p16 = 1 - 0.75 ** 16
    assert abs((trip >= 0).mean() - p16) < 4 * np.sqrt(p16 * (1 - p16) / trip.size)
    trip1 = ps.draw_triplets(win, b, 1, 0, 4000, 1)     # one attempt
    acc = (trip1 >= 0).mean()
    assert abs(acc - 0.25) < 4 * np.sqrt(0.25 * 0.75 / trip1.size)


def test_sampled_pose_step_keeps_the_true_pose_of_an_exact_window():
    """Exact flows (stored in FP32), true depth and poses: frame 1's observations are exact
    lookups, so every sample is the true pose up to the flows' FP32 rounding, and so is the
    mode; frame 2's carry bilinear-interpolation error as well."""
    w, win, b = exact_window(N=2, k=1)
    prm = dict(ps.DEFAULTS, samples=64)
    covs, info = ps.pose_sample_step(win, b, 0, prm)
    assert info[0, 0] == 64 and info[1, 0] >= 60
    np.testing.assert_allclose(b["pose"][0], w["pose_gt"][0], atol=1e-5)
    assert np.abs(b["pose"][1] - w["pose_gt"][1]).max() < 2e-3
    lam = np.linalg.eigvalsh(covs[0].reshape(6, 6))
    assert (lam >= prm["eps"] * (1 - 1e-9)).all()


def test_sampled_pose_step_recovers_perturbed_poses():
    """From perturbed initial poses the sampled step moves every frame towards the truth."""
    w, win, b = exact_window(N=3, k=2)
    b["pose"][...] = w["pose_init"]
    before = np.abs(b["pose"] - w["pose_gt"]).max(1)
    ps.pose_sample_step(win, b, 0, dict(ps.DEFAULTS, samples=128))
    after = np.abs(b["pose"] - w["pose_gt"]).max(1)
    print("pose error before", before, "after", after)
    assert (after < before).all() and after[0] < 1e-5
