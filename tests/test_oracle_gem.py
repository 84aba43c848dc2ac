"""Pins of the oracle's GEM steps: brute-force HMM enumeration, exhaustive inverse-depth
search, closed-form special cases, finite differences, fixed points and a linear-algebra
library."""
import itertools

import numpy as np
import pytest

from oracle import fisk, gem, geometry as geo
from paper_2104_06800_amd import synth


def brute_force_chain(e0, e1, gamma):
    """All 2^L labelings of one chain: marginals P(W_i = 1) and log Z."""
    L = len(e0)
    Z = 0.0
    m = np.zeros(L)
    for lab in itertools.product((0, 1), repeat=L):
        p = 0.5 * (e1[0] if lab[0] else e0[0])
        for i in range(1, L):
            p *= (gamma if lab[i] == lab[i - 1] else 1 - gamma) * (e1[i] if lab[i] else e0[i])
        Z += p
        m += p * np.array(lab)
    return m / Z, np.log(Z)


def small_window(N=3, H=12, W=16, tile=8, stride=4, seed_k=0, noise=True, **kw):
    w = synth.make_window(1, seed_k, noise=noise, H=H, W=W, N=N)
    win = dict(w["params"], tile=tile, coarse_stride=stride, **kw)
    return w, win


# ----------------------------------------------------------------------------- E-step
@pytest.mark.parametrize("gamma", [0.9, 0.6, 0.97])
def test_forward_backward_matches_enumeration(gamma):
    rng = np.random.default_rng(5)
    for L in (1, 2, 5, 11):
        e0 = rng.uniform(0.001, 0.01, size=(3, L))
        e1 = rng.uniform(0.0, 1.3, size=(3, L))
        q, logz = gem.forward_backward(e0, e1, gamma)
        for c in range(3):
            mq, lz = brute_force_chain(e0[c], e1[c], gamma)
            np.testing.assert_allclose(q[c], mq, atol=1e-12)
            assert logz[c] == pytest.approx(lz, rel=1e-12)


def test_forward_backward_limits():
    rng = np.random.default_rng(6)
    e0 = rng.uniform(0.001, 0.01, size=(4, 9))
    e1 = rng.uniform(0.0, 1.3, size=(4, 9))
    q, _ = gem.forward_backward(e0, e1, 0.5)          # independent nodes: per-node Bayes
    np.testing.assert_allclose(q, e1 / (e0 + e1), atol=1e-14)
    q, _ = gem.forward_backward(e0, e1, 1.0)          # frozen chain: two hypotheses
    a, b = np.prod(e0, 1), np.prod(e1, 1)
    np.testing.assert_allclose(q, np.repeat((b / (a + b))[:, None], 9, 1), atol=1e-12)


@pytest.mark.parametrize("level,d", [(1, 0), (1, 1), (1, 2), (0, 3), (0, 0)])
def test_spatial_estep_matches_enumeration(level, d):
    w, win = small_window(N=2, H=12, W=16, tile=8)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    gem.init_idepth(win, b)
    ll = gem.rigidness_fb(win, b, d, level)
    ww = gem.Window(win, b)
    lv = gem.Level(win, level)
    rho = b["idepth"].ravel()[lv.full]
    e0, e1, _ = ww.emissions(lv.u, lv.v, rho)
    out = b["rigid" if level == 1 else "rigid_coarse"].reshape(win["N"], -1)
    total = 0.0
    for g in gem.chains(win, level, d):
        for chain in g:
            if len(chain) > 12:
                continue
            for t in range(win["N"]):
                mq, lz = brute_force_chain(e0[t, chain], e1[t, chain], win["hmm_gamma"])
                np.testing.assert_allclose(out[t, chain], mq, atol=1e-12)
                total += lz
    if level == 1:
        assert ll == pytest.approx(total, rel=1e-12)


def test_temporal_estep_matches_enumeration():
    w, win = small_window(N=6, H=12, W=16, chain_axis=1)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    gem.init_idepth(win, b)
    ll = gem.rigidness_fb(win, b, 0, 1)
    ww = gem.Window(win, b)
    lv = gem.Level(win, 1)
    e0, e1, _ = ww.emissions(lv.u, lv.v, b["idepth"].ravel())
    tot = 0.0
    for j in range(0, lv.u.size, 7):
        mq, lz = brute_force_chain(e0[:, j], e1[:, j], win["hmm_gamma"])
        np.testing.assert_allclose(b["rigid"].reshape(6, -1)[:, j], mq, atol=1e-12)
    for j in range(lv.u.size):
        tot += brute_force_chain(e0[:, j], e1[:, j], win["hmm_gamma"])[1] if j % 97 == 0 else 0.0
    assert np.isfinite(ll) and np.isfinite(tot)


def test_chains_cover_every_pixel_once():
    _, win = small_window(H=37, W=70, tile=16, stride=4)
    for level in (0, 1):
        lv = gem.Level(win, level)
        for d in range(4):
            idx = np.concatenate([g.ravel() for g in gem.chains(win, level, d)])
            assert np.array_equal(np.sort(idx), np.arange(lv.h * lv.w))


# ----------------------------------------------------------------------------- M-step
def test_mstep_k3_is_running_best_along_chain():
    """With K = 3 (current, predecessor, coarse) a pass is a closed-form running best."""
    w, win = small_window(N=3, H=12, W=16, tile=8, n_candidates=3)
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    gem.init_idepth(win, b)
    rng = np.random.default_rng(3)
    b["rigid"][...] = rng.uniform(0, 1, b["rigid"].shape)
    b["idepth_coarse"][...] = rng.uniform(0.05, 1.0, b["idepth_coarse"].shape)
    rho0 = b["idepth"].copy()
    gem.depth_update(win, b, 1, 1)
    ww = gem.Window(win, b)
    s = win["coarse_stride"]
    hc, wc = gem.lattice_shape(win["H"], win["W"], s)
    for g in gem.chains(win, 1, 1):
        for chain in g:
            prev = None
            for i, p in enumerate(chain):
                v, u = divmod(int(p), win["W"])
                c = [rho0.flat[p], rho0.flat[p] if i == 0 else prev,
                     b["idepth_coarse"][min(v // s, hc - 1), min(u // s, wc - 1)]]
                E = [ww.energy(np.array([u]), np.array([v]), np.array([[x]]),
                               b["rigid"].reshape(3, -1)[:, [p]], np.zeros((0, 1)))[0, 0] for x in c]
                best = c[0]
                Eb = E[0]
                for x, e in zip(c[1:], E[1:]):
                    if e < Eb:
                        best, Eb = x, e
                assert b["idepth"].flat[p] == best
                prev = best


def test_mstep_ties_keep_current_value():
    w, win = small_window(N=3)
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    gem.init_idepth(win, b)
    rho0 = b["idepth"].copy()
    b["rigid"][...] = 0.0                  # every candidate costs 0: all slots tie
    gem.depth_update(win, b, 0, 1)
    assert np.array_equal(b["idepth"], rho0)


def test_mstep_reaches_exhaustive_minimum():
    """With q and poses fixed E_j is separable per pixel, so a 2e4-point grid search refined
    by golden section gives each pixel's minimum.  After 20 passes with K = 32 GEM's value is
    within 1e-4 of it on >= 99% of pixels and within 1e-2 everywhere (the search is
    stochastic and refines at a relative step of at least 0.5%)."""
    w, win = small_window(N=3, H=12, W=16, tile=8, n_candidates=32)
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    gem.init_idepth(win, b)
    gem.rigidness_fb(win, b, 0, 1)
    q = b["rigid"].copy()
    for it in range(20):
        b["rigid_coarse"][...] = q[:, win["coarse_stride"] // 2::win["coarse_stride"],
                                   win["coarse_stride"] // 2::win["coarse_stride"]]
        gem.depth_update(win, b, it, 0)
        b["rigid"][...] = q
        gem.depth_update(win, b, it, 1)
    ww = gem.Window(win, b)
    lv = gem.Level(win, 1)
    qf = q.reshape(3, -1)
    grid = np.linspace(win["idepth_min"], win["idepth_max"], 20000)
    Eg = ww.energy(lv.u, lv.v, np.repeat(grid[None], lv.u.size, 0), qf, np.zeros((0, lv.u.size)))
    k = np.argmin(Eg, 1)
    lo = grid[np.maximum(k - 1, 0)]
    hi = grid[np.minimum(k + 1, grid.size - 1)]
    gr = (np.sqrt(5) - 1) / 2
    for _ in range(40):                                 # golden-section refinement
        a = hi - gr * (hi - lo)
        c = lo + gr * (hi - lo)
        Ea = ww.energy(lv.u, lv.v, a[:, None], qf, np.zeros((0, lv.u.size)))[:, 0]
        Ec = ww.energy(lv.u, lv.v, c[:, None], qf, np.zeros((0, lv.u.size)))[:, 0]
        hi = np.where(Ea < Ec, c, hi)
        lo = np.where(Ea < Ec, lo, a)
    Emin = np.minimum(Eg.min(1), ww.energy(lv.u, lv.v, (0.5 * (lo + hi))[:, None], qf,
                                           np.zeros((0, lv.u.size)))[:, 0])
    Egem = ww.energy(lv.u, lv.v, b["idepth"].ravel()[:, None], qf, np.zeros((0, lv.u.size)))[:, 0]
    # nothing beats the exhaustive minimum by more than the grid spacing can hide: where a
    # term turns invalid the energy steps, and the infimum sits on the step
    tol = 1e-4 * np.maximum(1.0, np.abs(Emin))
    assert (Egem >= Emin - tol).all()
    frac = np.mean(Egem <= Emin + tol)
    assert frac >= 0.99, frac
    assert (Egem <= Emin + 1e-2).all()


def test_gem_fixed_point_single_frame():
    """Noise-free scene, N = 1, start at the true depth and pose: depth unchanged bit for
    bit (ties keep the current value), pose within float32 flow-storage rounding."""
    w = synth.make_window(1, 4, noise=False, N=1)
    win = w["params"]
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    b["idepth"][...] = w["idepth_gt"]
    gem.gem_step(win, b, 0)
    gem.gem_step(win, b, 1)
    assert np.array_equal(b["idepth"], w["idepth_gt"])
    assert np.abs(b["pose"] - w["pose_gt"]).max() < 1e-7


def test_gem_with_fixed_true_poses_recovers_depth():
    """Noise-free flows, true poses held fixed: E and M steps alone recover the depth
    (border pixels whose track leaves the image excepted)."""
    w = synth.make_window(1, 1, noise=False)
    win = w["params"]
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"])
    gem.init_idepth(win, b)
    for it in range(5):
        for lvl in (0, 1):
            gem.rigidness_fb(win, b, it, lvl)
            gem.depth_update(win, b, it, lvl)
    e = np.abs(b["idepth"] - w["idepth_gt"]) / w["idepth_gt"]
    assert np.median(e) < 0.003
    assert np.mean(e < 0.02) > 0.9


# ----------------------------------------------------------------------------- pose
def test_pose_score_gradient_and_hessian_by_finite_differences():
    w, win = small_window(N=3, H=24, W=32, tile=8)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    b["idepth"][...] = w["idepth_gt"]
    rng = np.random.default_rng(9)
    b["rigid"][...] = rng.uniform(0.2, 1.0, b["rigid"].shape)
    for t in (1, 3):
        p0 = b["pose"][t - 1].copy()
        row = gem.pose_score(win, b, t, p0[None])[0]
        H, g = gem.unpack_normal_equations(row)
        for i in range(6):
            d = np.zeros(6)
            d[i] = 1e-6
            Ep = gem.pose_score(win, b, t, geo.left_update(p0, d)[None])[0, 0]
            Em = gem.pose_score(win, b, t, geo.left_update(p0, -d)[None])[0, 0]
            assert (Ep - Em) / 2e-6 == pytest.approx(2 * g[i], rel=1e-5, abs=1e-6)
        assert np.all(np.linalg.eigvalsh(H) >= -1e-9 * np.trace(H))


def test_pose_score_counts_only_reprojections_inside_frame_t():
    """Brute force per pixel: a term is valid iff its point is in front of both cameras, the
    flow sample of frame t-1 exists, and the reprojection into frame t lies in the image."""
    w, win = small_window(N=2, H=20, W=28, tile=8)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    b["idepth"][...] = w["idepth_gt"]
    b["rigid"][...] = 0.7
    fx, fy, cx, cy = win["fx"], win["fy"], win["cx"], win["cy"]
    t = 2
    # a candidate that rotates part of the image out of frame t
    cand = geo.left_update(b["pose"][t - 1], np.array([0.0, 0.25, 0.0, 0.0, 0.0, 0.0]))
    Rp, tp = geo.pose_rt(b["pose"][t - 2])
    Rc, tc = geo.pose_rt(cand)
    count = seen = 0
    for v in range(win["H"]):
        for u in range(win["W"]):
            X = np.array([(u - cx) / fx, (v - cy) / fy, 1.0]) / w["idepth_gt"][v, u]
            Qp, Qc = Rp @ X + tp, Rc @ X + tc
            if Qp[2] <= 0 or Qc[2] <= 0:
                continue
            pu, pv = fx * Qp[0] / Qp[2] + cx, fy * Qp[1] / Qp[2] + cy
            if not (0 <= pu <= win["W"] - 1 and 0 <= pv <= win["H"] - 1):
                continue
            seen += 1
            cu, cv = fx * Qc[0] / Qc[2] + cx, fy * Qc[1] / Qc[2] + cy
            count += (0 <= cu <= win["W"] - 1) and (0 <= cv <= win["H"] - 1)
    row = gem.pose_score(win, b, t, cand[None])[0]
    assert 0 < count < seen - 20          # the rule removes a good share of the terms
    assert row[28] == count


def test_pose_score_of_a_view_away_from_the_scene_is_uninformative():
    w, win = small_window(N=2, H=20, W=28, tile=8)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    b["idepth"][...] = w["idepth_gt"]
    rng = np.random.default_rng(3)
    b["rigid"][...] = rng.uniform(0.0, 1.0, b["rigid"].shape)
    cand = geo.left_update(b["pose"][0], np.array([0.0, np.pi / 2, 0.0, 0.0, 0.0, 0.0]))
    row = gem.pose_score(win, b, 1, cand[None])[0]
    assert row[28] == 0 and np.all(row[1:28] == 0)
    assert row[0] == pytest.approx(np.log(2) * b["rigid"][0].sum(), rel=1e-12)


def test_pose_jacobian_by_finite_differences():
    win = synth.default_params(10, 12, 1, (30.0, 30.0, 6.0, 5.0))
    rng = np.random.default_rng(4)
    Q = rng.uniform([-1, -1, 2], [1, 1, 4], size=(5, 3))
    rho = rng.uniform(0.2, 0.8, 5)
    J = gem._jac_rows(Q, rho, 30.0, 31.0)
    for i in range(6):
        d = np.zeros(6)
        d[i] = 1e-7
        def proj(dd):
            E = geo.exp_so3(dd[:3])
            Qn = Q @ E.T + rho[:, None] * dd[3:]
            return np.stack([30.0 * Qn[:, 0] / Qn[:, 2], 31.0 * Qn[:, 1] / Qn[:, 2]], -1)
        fd = (proj(d) - proj(-d)) / 2e-7
        np.testing.assert_allclose(J[:, :, i], fd, rtol=1e-6, atol=1e-6)
    del win


def test_cholesky_matches_numpy_and_detects_singular():
    rng = np.random.default_rng(8)
    for _ in range(20):
        A = rng.normal(size=(6, 6))
        A = A @ A.T + 0.1 * np.eye(6)
        b = rng.normal(size=6)
        np.testing.assert_allclose(gem.cholesky_solve(A, b), np.linalg.solve(A, b), rtol=1e-10)
    A = np.diag([1.0, 2.0, 0.0, 3.0, 1.0, 1.0])
    assert gem.cholesky_solve(A, np.ones(6)) is None
    assert gem.cholesky_solve(-np.eye(6), np.ones(6)) is None
    assert gem.cholesky_solve(np.zeros((6, 6)), np.ones(6)) is None


def test_pose_step_converges_to_truth():
    w = synth.make_window(1, 2, noise=False)
    win = w["params"]
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    b["idepth"][...] = w["idepth_gt"]
    b["rigid"][...] = 1.0
    for _ in range(3):
        gem.pose_step(win, b)
    # frame 1 uses an exact flow lookup; later frames carry bilinear-interpolation error
    assert np.abs(b["pose"][0] - w["pose_gt"][0]).max() < 1e-7
    assert np.abs(b["pose"] - w["pose_gt"]).max() < 5e-5


# ----------------------------------------------------------------------------- priors, confidence
def test_prior_alone_pins_depth():
    """No flow weight (q = 0) and an identity-pose prior: the prior value wins when it is a
    candidate, and a pass from elsewhere never increases the prior energy."""
    w, win = small_window(N=3, P=1)
    H, W = win["H"], win["W"]
    rng = np.random.default_rng(11)
    prior = rng.uniform(0.1, 0.9, (1, H, W))
    prior[0, 3, 4] = np.nan
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"], prior, np.zeros((1, 6)))
    b["rigid"][...] = 0.0
    b["idepth"][...] = prior[0]
    b["idepth"][3, 4] = 0.5
    gem.depth_update(win, b, 0, 1)
    assert np.array_equal(b["idepth"], np.where(np.isnan(prior[0]), 0.5, prior[0]))
    b["idepth"][...] = np.clip(prior[0] * 1.3, 0.02, 1.25)
    b["idepth"][3, 4] = 0.5
    ww = gem.Window(win, b)
    lv = gem.Level(win, 1)
    before = np.abs(b["idepth"].ravel() - prior[0].ravel())
    gem.depth_update(win, b, 5, 1)
    after = np.abs(b["idepth"].ravel() - prior[0].ravel())
    ok = np.isfinite(before)
    assert (after[ok] <= before[ok] + 1e-15).all()
    assert b["idepth"][3, 4] == 0.5                      # hole: no term, all slots tie
    del ww, lv


def test_confidence_reduces_to_per_node_bayes():
    """gamma = 1/2 and no priors: C = mean_t L1/(L0 + L1) with L1 from scipy's Fisk law."""
    from scipy import stats
    w, win = small_window(N=3, hmm_gamma=0.5)
    b = gem.alloc_buffers(win, w["flow"], w["pose_init"])
    gem.init_idepth(win, b)
    st = gem.finalize(win, b, 0)
    ww = gem.Window(win, b)
    lv = gem.Level(win, 1)
    r2, ok = ww.flow_residuals(lv.u, lv.v, b["idepth"].ravel())
    r = np.sqrt(r2)
    a = win["fisk_alpha"]
    L1 = np.where(r > 0, stats.fisk.pdf(r, c=2.0, scale=a) / (2 * np.pi * np.where(r > 0, r, 1)),
                  1 / (np.pi * a * a))
    L1 = np.where(ok, L1, win["outlier_density"])
    C = (L1 / (L1 + win["outlier_density"])).mean(0)
    np.testing.assert_allclose(b["conf"].ravel(), C, atol=1e-12)
    assert st[5] == pytest.approx(C.sum(), rel=1e-12)
    assert st[2] + st[3] == 3 * lv.u.size


# ----------------------------------------------------------------------------- prior transfer (Eq. 3)
def _prior_window(H, W, prior_pose, prior_map, f=40.0):
    w, win = small_window(N=1, H=H, W=W, P=1)
    win = dict(win, fx=f, fy=f, cx=(W - 1) / 2 + 0.3, cy=(H - 1) / 2 - 0.2)
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"], prior_map[None], np.asarray(prior_pose)[None])
    return win, gem.Window(win, b)


@pytest.mark.parametrize("tz", [0.8, -0.35])
def test_prior_transfer_pure_forward_translation_closed_form(tz):
    """Prior camera displaced by t_z along the optical axis: the point of pixel j at inverse
    depth rho lies at depth 1/rho + t_z in the prior camera, so 1/phi_z = rho/(1 + rho t_z)
    and it projects to c + (j - c)/(1 + rho t_z); the prior value is read at the nearest
    pixel of that point (Eq. 3: l = pi(theta^j, T^_k), compared with 1/phi_z)."""
    H, W = 30, 40
    yy, xx = np.mgrid[0:H, 0:W]
    prior = 0.1 + 0.003 * xx + 0.0011 * yy          # distinct value at every pixel
    win, ww = _prior_window(H, W, [0, 0, 0, 0, 0, tz], prior)
    rng = np.random.default_rng(21)
    u = rng.integers(0, W, 400)
    v = rng.integers(0, H, 400)
    rho = rng.uniform(0.05, 1.0, 400)
    z, ok = ww.prior_z(0, u, v, rho)
    D = 1.0 + rho * tz
    front = D > 0
    lx = np.floor((u - win["cx"]) / np.where(front, D, 1) + win["cx"] + 0.5)
    ly = np.floor((v - win["cy"]) / np.where(front, D, 1) + win["cy"] + 0.5)
    inside = front & (lx >= 0) & (lx <= W - 1) & (ly >= 0) & (ly <= H - 1)
    assert inside.sum() > 100 and (tz > 0 or (~inside).sum() > 5)
    np.testing.assert_array_equal(ok, inside)
    rh = 0.1 + 0.003 * lx + 0.0011 * ly
    want = (rh - rho / D) / (win["prior_sigma_rel"] * rh)
    np.testing.assert_allclose(z[inside], want[inside], rtol=1e-12, atol=1e-12)
    assert (z[~inside] == 0).all()


def test_prior_transfer_rotated_camera_matches_ray_caster():
    """A rotated and translated prior camera looking at two planes that are fronto-parallel
    to it (one in front of the other), its inverse-depth map ray-cast by the input
    generator: at the true reference inverse depth every pixel whose transfer lands inside
    one plane's image region has z = 0 to rounding, since the prior value is constant
    over each plane.  A tilted third plane bounds z by the map's gradient over half a
    pixel (nearest sampling).  A wrong direction of T^ or of the depth transfer breaks
    both."""
    H, W, f = 36, 48, 40.0
    intr = (f, f, (W - 1) / 2 + 0.3, (H - 1) / 2 - 0.2)
    Rk = synth._rot(np.deg2rad([3.0, -4.0, 2.0]))
    tk = np.array([0.12, -0.05, 0.3])
    axis = Rk[2]                                    # prior camera's optical axis, world frame
    cam_c = -Rk.T @ tk                              # prior camera centre, world frame
    planes_n, planes_d = [], []
    for depth in (4.0, 9.0):                        # fronto-parallel to the prior camera
        planes_n.append(-axis)
        planes_d.append(-(axis @ cam_c + depth))
    scene = synth.Scene(planes_n=np.array(planes_n), planes_d=np.array(planes_d),
                        quads=[synth._quad([1.0, 0.3, 3.0], 25.0, 10.0, 0.9, 0.6)])
    z_ref, obj_ref, _ = synth._raycast(scene, 0, H, W, intr, (np.eye(3), np.zeros(3)))
    z_k, obj_k, _ = synth._raycast(scene, 0, H, W, intr, (Rk, tk))
    pose_k = synth._as6((Rk, tk))
    win, ww = _prior_window(H, W, pose_k, 1.0 / z_k, f=f)
    win.update(cx=intr[2], cy=intr[3])
    ww = gem.Window(win, ww.b)
    V, U = np.mgrid[0:H, 0:W]
    u, v = U.ravel(), V.ravel()
    rho = 1.0 / z_ref.ravel()
    z, ok = ww.prior_z(0, u, v, rho)
    # where does each reference point land in the prior camera (generator's projection)
    X = synth._rays(H, W, *intr, (np.eye(3), np.zeros(3)))[1].reshape(-1, 3) * z_ref.ravel()[:, None]
    px, py, _ = synth._project(X, (Rk, tk), intr)
    lx, ly = np.floor(px + 0.5).astype(int), np.floor(py + 0.5).astype(int)
    inside = (lx >= 1) & (lx <= W - 2) & (ly >= 1) & (ly <= H - 2)
    assert ok[inside].all()
    lxc, lyc = np.clip(lx, 0, W - 1), np.clip(ly, 0, H - 1)
    same_obj = obj_k[lyc, lxc] == obj_ref.ravel()   # the prior pixel sees the same surface
    nb = np.stack([obj_k[np.clip(lyc + dy, 0, H - 1), np.clip(lxc + dx, 0, W - 1)]
                   for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    interior = inside & same_obj & (nb == obj_k[lyc, lxc]).all(0)
    flat = interior & (obj_ref.ravel() < 100)
    tilted = interior & (obj_ref.ravel() >= 100)
    assert flat.sum() > 300 and tilted.sum() > 30
    assert np.abs(z[flat]).max() < 1e-9
    rk = 1.0 / z_k
    gx = np.abs(rk[lyc, np.clip(lxc + 1, 0, W - 1)] - rk[lyc, lxc])
    gy = np.abs(rk[np.clip(lyc + 1, 0, H - 1), lxc] - rk[lyc, lxc])
    diff = np.abs(z * win["prior_sigma_rel"] * rk[lyc, lxc])   # |rho^(l) - 1/phi_z|
    assert (diff[tilted] <= 0.5 * (gx + gy)[tilted] * 1.01 + 1e-12).all()
    assert np.abs(z[tilted]).max() > 1e-6        # nearest sampling is visible there


# ----------------------------------------------------------------------------- initial depth from a prior
@pytest.mark.parametrize("tz", [0.8, -0.35])
def test_prior_bootstrap_forward_translation_closed_form(tz):
    """A fronto-parallel plane at depth Z seen by a prior camera displaced by t_z along the
    optical axis: its prior map is 1/(Z + t_z) everywhere, and the start value must be the
    true 1/Z at every pixel whose transfer stays inside the prior image (all of them for
    t_z > 0; for t_z < 0 the border pixels land outside and stay random)."""
    H, W, Z = 30, 40, 3.0
    prior = np.full((H, W), 1.0 / (Z + tz))
    win, ww = _prior_window(H, W, [0, 0, 0, 0, 0, tz], prior)
    rho, ok = gem.prior_bootstrap(win, ww.b)
    np.testing.assert_allclose(rho[ok], 1.0 / Z, rtol=1e-13)
    if tz > 0:
        assert ok.all()
    else:
        # a point at inverse depth r lands at c + (j - c) / (1 + r t_z); both rounds must land
        # inside: the first from the prior's own value 1/(Z + t_z), the second from 1/Z
        V, U = np.mgrid[0:H, 0:W]
        inside = np.ones((H, W), dtype=bool)
        for r in (1.0 / (Z + tz), 1.0 / Z):
            D = 1.0 + r * tz
            lx = np.floor((U - win["cx"]) / D + win["cx"] + 0.5)
            ly = np.floor((V - win["cy"]) / D + win["cy"] + 0.5)
            inside &= (lx >= 0) & (lx <= W - 1) & (ly >= 0) & (ly <= H - 1)
        assert 50 < (~inside).sum() < inside.sum()
        np.testing.assert_array_equal(ok, inside)


def test_prior_bootstrap_two_rounds_on_a_varying_map():
    """Forward translation t_z = 0.6 over a prior map that varies per pixel: each round reads
    the map where the previous value lands, c + (j - c) / (1 + r t_z), and solves
    rho = rho^(l) / (1 - rho^(l) t_z) (r_3 . x~ = 1 without rotation); the second round
    starts from the first round's value."""
    H, W, tz = 30, 40, 0.6
    yy, xx = np.mgrid[0:H, 0:W]
    prior = 0.2 + 0.004 * xx + 0.002 * yy
    win, ww = _prior_window(H, W, [0, 0, 0, 0, 0, tz], prior)
    rho, ok = gem.prior_bootstrap(win, ww.b)
    assert ok.all()
    r = prior.copy()
    for _ in range(2):
        D = 1.0 + r * tz
        lx = np.floor((xx - win["cx"]) / D + win["cx"] + 0.5).astype(int)
        ly = np.floor((yy - win["cy"]) / D + win["cy"] + 0.5).astype(int)
        rh = prior[ly, lx]
        r = rh / (1.0 - rh * tz)
    np.testing.assert_allclose(rho, r, rtol=1e-13)
    one, _ = gem.prior_bootstrap(win, ww.b, rounds=1)
    assert (one != rho).sum() > 50           # the second round moves many pixels


def test_prior_bootstrap_rotated_camera_matches_ray_caster():
    """A rotated and translated prior camera in front of two planes fronto-parallel to it,
    its inverse-depth map ray-cast by the input generator: the start value equals the true
    reference inverse depth to rounding wherever the transfer lands well inside the plane
    region the reference pixel sees (the prior is constant there, so any landing pixel on
    that plane gives the exact solution).  A wrong direction of T^, a dropped r_3 . x~
    factor or a wrong sign of t_z breaks it."""
    H, W, f = 36, 48, 40.0
    intr = (f, f, (W - 1) / 2 + 0.3, (H - 1) / 2 - 0.2)
    Rk = synth._rot(np.deg2rad([3.0, -4.0, 2.0]))
    tk = np.array([0.12, -0.05, 0.3])
    axis, cam_c = Rk[2], -Rk.T @ tk
    scene = synth.Scene(planes_n=np.array([-axis, -axis]),
                        planes_d=np.array([-(axis @ cam_c + 4.0), -(axis @ cam_c + 9.0)]),
                        quads=[synth._quad([1.0, 0.3, 3.0], 25.0, 10.0, 0.9, 0.6)])
    z_ref, obj_ref, _ = synth._raycast(scene, 0, H, W, intr, (np.eye(3), np.zeros(3)))
    z_k, obj_k, _ = synth._raycast(scene, 0, H, W, intr, (Rk, tk))
    win, ww = _prior_window(H, W, synth._as6((Rk, tk)), 1.0 / z_k, f=f)
    win.update(cx=intr[2], cy=intr[3])
    rho, ok = gem.prior_bootstrap(win, gem.Window(win, ww.b).b)
    X = synth._rays(H, W, *intr, (np.eye(3), np.zeros(3)))[1].reshape(-1, 3) * z_ref.ravel()[:, None]
    px, py, _ = synth._project(X, (Rk, tk), intr)
    lx, ly = np.floor(px + 0.5).astype(int), np.floor(py + 0.5).astype(int)
    lxc, lyc = np.clip(lx, 0, W - 1), np.clip(ly, 0, H - 1)
    inside = (lx >= 2) & (lx <= W - 3) & (ly >= 2) & (ly <= H - 3)
    nb = np.stack([obj_k[np.clip(lyc + dy, 0, H - 1), np.clip(lxc + dx, 0, W - 1)]
                   for dy in range(-2, 3) for dx in range(-2, 3)])
    flat = inside & (obj_ref.ravel() < 100) & (nb == obj_ref.ravel()).all(0)
    assert flat.sum() > 300
    # the start at the same pixel lands near the true l; every such pixel resolves exactly
    good = flat & ok.ravel()
    assert good.sum() >= 0.95 * flat.sum()
    np.testing.assert_allclose(rho.ravel()[good], 1.0 / z_ref.ravel()[good], rtol=1e-10)


def test_init_idepth_uses_prior_where_it_resolves():
    """Identity prior pose: the start is the prior clamped to [rho_min, rho_max] at every
    finite positive prior pixel and the random start (bit for bit) at holes; init_random
    restores the random start everywhere."""
    H, W = 20, 24
    rng = np.random.default_rng(3)
    prior = rng.uniform(0.0, 1.6, (H, W))
    prior[rng.uniform(size=(H, W)) < 0.2] = np.nan
    prior[0, :3] = [0.0, -0.2, np.inf]
    win, ww = _prior_window(H, W, np.zeros(6), prior)
    win = dict(win, idepth_min=0.05, idepth_max=1.25)
    b = ww.b
    gem.init_idepth(win, b)
    start = b["idepth"].copy()
    gem.init_idepth(dict(win, P=0), b)
    rand = b["idepth"].copy()
    gem.init_idepth(dict(win, init_random=1), b)
    np.testing.assert_array_equal(b["idepth"], rand)
    good = np.isfinite(prior) & (prior > 0)
    np.testing.assert_array_equal(start[good], np.clip(prior[good], 0.05, 1.25))
    np.testing.assert_array_equal(start[~good], rand[~good])
    assert (~good).sum() > 50 and (prior[good] > 1.25).sum() > 10 and (prior[good] < 0.05).sum() > 5


# ----------------------------------------------------------------------------- empirical disparity prior model
@pytest.mark.parametrize("beta", [1.0, 0.7])
def test_disparity_model_matches_fisk_law(beta):
    """Inlier density of a signed disparity residual: the log-logistic law of |r| halved
    (scipy's fisk), a density on the line; the MIE cost and posterior from their
    definitions."""
    from scipy import integrate, stats
    a, D = 0.6, 64.0
    r = np.array([-5.0, -0.7, -0.01, 0.02, 0.3, 1.1, 9.0])
    p1 = stats.fisk.pdf(np.abs(r), c=beta, scale=a) / 2
    p0 = 1.0 / D
    np.testing.assert_allclose(fisk.disparity_log_ratio(r, a, beta, D), np.log(p0 / p1), rtol=1e-12)
    np.testing.assert_allclose(fisk.disparity_prior_term(r, a, beta, D), -np.log(p1 / (p0 + p1)), rtol=1e-12)
    pi = 0.35
    np.testing.assert_allclose(fisk.disparity_prior_posterior(r, a, beta, D, pi), pi * p1 / (pi * p1 + (1 - pi) * p0),
                               rtol=1e-12)
    # mass on the line: the law's CDF z^b / (1 + z^b); below |r| = 1e-3 a the density of a
    # shape < 1 is floored, so the integral starts past the floor there
    lo = 0.0 if beta == 1.0 else 2e-3 * a
    half = integrate.quad(lambda x: np.exp(-fisk.disparity_log_ratio(x, a, beta, D)) / D, lo, np.inf, limit=200)[0]
    z = lo / a
    assert 2 * half == pytest.approx(1.0 - z ** beta / (1 + z ** beta), rel=1e-6)


def test_disparity_transfer_closed_form():
    """The transfer under pure forward translation with the disparity model: z is the
    disparity residual fb (rho^(l) - rho / (1 + rho t_z))."""
    H, W, tz, fb = 30, 40, -0.35, 389.0
    yy, xx = np.mgrid[0:H, 0:W]
    prior = 0.1 + 0.003 * xx + 0.0011 * yy
    win, ww = _prior_window(H, W, [0, 0, 0, 0, 0, tz], prior)
    win.update(prior_model=1, prior_disp_scale=fb, prior_fisk_beta=1.0)
    ww = gem.Window(win, ww.b)
    rng = np.random.default_rng(23)
    u, v, rho = rng.integers(0, W, 300), rng.integers(0, H, 300), rng.uniform(0.05, 1.0, 300)
    z, ok = ww.prior_z(0, u, v, rho)
    D = 1.0 + rho * tz
    lx = np.floor((u - win["cx"]) / D + win["cx"] + 0.5)
    ly = np.floor((v - win["cy"]) / D + win["cy"] + 0.5)
    inside = (lx >= 0) & (lx <= W - 1) & (ly >= 0) & (ly <= H - 1)
    np.testing.assert_array_equal(ok, inside)
    np.testing.assert_allclose(z[inside], fb * (0.1 + 0.003 * lx + 0.0011 * ly - rho / D)[inside], rtol=1e-12)


def test_disparity_prior_alone_pins_depth():
    """No flow weight (q = 0), the disparity model with an identity-pose prior: every pixel
    whose prior value is among its candidates takes it (the density peaks at r = 0), and a
    pass from elsewhere never moves a pixel away from its prior."""
    w, win = small_window(N=3, P=1)
    win.update(prior_model=1, prior_disp_scale=200.0, prior_fisk_beta=1.0, prior_sigma_rel=0.5,
               prior_uniform_rel=100.0)
    H, W = win["H"], win["W"]
    rng = np.random.default_rng(12)
    prior = rng.uniform(0.1, 0.9, (1, H, W))
    b = gem.alloc_buffers(win, w["flow"], w["pose_gt"], prior, np.zeros((1, 6)))
    b["rigid"][...] = 0.0
    b["idepth"][...] = prior[0]
    gem.depth_update(win, b, 0, 1)
    assert np.array_equal(b["idepth"], prior[0])
    b["idepth"][...] = np.clip(prior[0] * 1.3, 0.02, 1.25)
    before = np.abs(b["idepth"] - prior[0])
    gem.depth_update(win, b, 5, 1)
    assert (np.abs(b["idepth"] - prior[0]) <= before + 1e-15).all()
