"""Uncertainty-aware pose estimation by Monte-Carlo P3P sampling, FP64 (test
infrastructure).

Sec. III-A "Uncertainty-aware Pose Estimation" (its sampling equation): with the other
parameters fixed, the posterior of frame t's pose is approximated by S pose samples, each
solved from a P3P instance (three pixels' 3D points and their observed image positions in
frame t) and widened by a fixed covariance Sigma; the pose is the mode of that mixture,
found by meanshift with a Gaussian kernel in the pose's Lie algebra; the pose uncertainty
Sigma_t is fitted to the samples starting from the mode, discarding samples outside 3 sigma,
with every eigenvalue held above an epsilon.

Readings (the paper leaves them to the VOLDOR framework and to the P3P solver it cites):
  * triplets are drawn with probability proportional to the rigidness posterior q_t^j by
    rejection: a Philox draw picks a pixel uniformly, a second accepts it when u < q_t^j and
    the pixel has a usable depth and observation; up to `tries` attempts per point (a
    sample whose point finds none is void).  Philox counter (sample g, k * tries + r for
    point k and attempt r, (it << 8) | (t << 4) | 2, window id); the pixel is
    (x0 * H W) >> 32 of output word 0, the acceptance uniform (x1 >> 8) 2^-24 of word 1;
  * the 3D point is x~_j / rho_j in the reference camera; its observation in frame t is
    o_t = p_{t-1} + X_t(p_{t-1}) as in the GEM steps (p_{t-1} under the current pose of
    frame t-1), turned into a unit bearing K^-1 [o_t, 1];
  * P3P is solved from the law of cosines of the three rays (Grunert's elimination to a
    quartic in the ratio of two ray lengths); of a triplet's real solutions the sample keeps
    the one nearest the frame's current pose in the kernel's metric; the rigid motion of a
    solution follows from the three point pairs by orthonormal triads;
  * the Lie-algebra coordinates of a pose T about a pose M are the left-update chart of the
    GEM pose step: (log(R_T R_M^T), t_T - R_T R_M^T t_M), inverse (w, v) ->
    (exp([w]x) R_M, exp([w]x) t_M + v);
  * the kernel covariance is diag(sigma_w^2 I, (sigma_t_rel |t|)^2 I) about the current
    pose; meanshift starts at the current pose and moves by the kernel-weighted mean of the
    samples' coordinates about the current mode until the step is below 1e-12 in kernel
    units (at most 100 steps);
  * the covariance fit starts from the mode and the kernel covariance: samples within
    Mahalanobis distance 3 of the current mean (about the mode) give the next mean and
    covariance, eigenvalues floored at eps; it stops when the inlier set repeats, after 20
    rounds, or below 7 inliers (keeping the previous fit).  The covariance of the inliers
    (1/n) is divided by KAPPA = P(chi2_8 <= 9) / P(chi2_6 <= 9), the share of a 6-D
    Gaussian's variance inside its own 3-sigma region: without it every round would shrink
    a Gaussian's fit, towards 0.43 times its covariance.  The frame's pose becomes the mode.
"""
import numpy as np
from numpy.polynomial import polynomial as P

from . import geometry as geo
from . import philox

PURPOSE_POSE = 2
# P(chi2_k <= 9) for even k = 2m is 1 - exp(-9/2) sum_{i<m} (9/2)^i / i!
_E = np.exp(-4.5)
KAPPA = (1.0 - _E * (1.0 + 4.5 + 4.5 ** 2 / 2 + 4.5 ** 3 / 6)) / (1.0 - _E * (1.0 + 4.5 + 4.5 ** 2 / 2))


# --------------------------------------------------------------------------- #
# P3P
# --------------------------------------------------------------------------- #
def rigid_from_triads(X, C):
    """(R, t) with C_i = R X_i + t for three exact point pairs (rows), from the orthonormal
    frames their triangles span."""
    def triad(Y):
        e1 = Y[1] - Y[0]
        e1 = e1 / np.linalg.norm(e1)
        e3 = np.cross(Y[1] - Y[0], Y[2] - Y[0])
        e3 = e3 / np.linalg.norm(e3)
        return np.stack([e1, np.cross(e3, e1), e3], axis=1)      # columns
    R = triad(C) @ triad(X).T
    return R, C[0] - R @ X[0]


def p3p(X, f):
    """All rigid motions (R, t), C = R X + t, that put the three points X [3][3] on the
    three unit bearings f [3][3] at positive depth (law of cosines, Grunert's quartic)."""
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    a2 = np.sum((X[1] - X[2]) ** 2)
    b2 = np.sum((X[0] - X[2]) ** 2)
    c2 = np.sum((X[0] - X[1]) ** 2)
    ca, cb, cg = f[1] @ f[2], f[0] @ f[2], f[0] @ f[1]
    # s2 = u s1, s3 = v s1:  b^2 (u^2 + v^2 - 2uv ca) = a^2 (1 + v^2 - 2v cb)
    #                        b^2 (1 + u^2 - 2u cg)    = c^2 (1 + v^2 - 2v cb)
    # their difference is linear in u: u = Nu(v) / Du(v); the second, times Du^2, is a quartic
    Nu = np.array([a2 - c2 + b2, -2.0 * (a2 - c2) * cb, a2 - c2 - b2])
    Du = np.array([2.0 * b2 * cg, -2.0 * b2 * ca])
    lhs = b2 * P.polyadd(P.polyadd(P.polymul(Du, Du), P.polymul(Nu, Nu)), -2.0 * cg * P.polymul(Nu, Du))
    rhs = c2 * P.polymul([1.0, -2.0 * cb, 1.0], P.polymul(Du, Du))
    quartic = P.polysub(lhs, rhs)
    if not np.all(np.isfinite(quartic)) or np.abs(quartic).max() == 0:
        return []
    roots = P.polyroots(np.trim_zeros(quartic, "b"))
    dq = P.polyder(quartic)
    out = []
    for r in roots:
        if abs(r.imag) > 1e-9 * max(1.0, abs(r.real)):
            continue
        v = r.real
        for _ in range(3):                 # Newton polish of the eigenvalue-based root
            dv = P.polyval(v, dq)
            if dv == 0:
                break
            v = v - P.polyval(v, quartic) / dv
        du = P.polyval(v, Du)
        if v <= 0 or du == 0:
            continue
        u = P.polyval(v, Nu) / du
        den = 1.0 + v * v - 2.0 * v * cb
        if u <= 0 or den <= 0:
            continue
        s = np.sqrt(b2 / den) * np.array([1.0, u, v])
        for _ in range(2):                 # Newton on the three law-of-cosines equations
            F = np.array([s[1] ** 2 + s[2] ** 2 - 2 * s[1] * s[2] * ca - a2,
                          s[0] ** 2 + s[2] ** 2 - 2 * s[0] * s[2] * cb - b2,
                          s[0] ** 2 + s[1] ** 2 - 2 * s[0] * s[1] * cg - c2])
            J = np.array([[0.0, 2 * s[1] - 2 * s[2] * ca, 2 * s[2] - 2 * s[1] * ca],
                          [2 * s[0] - 2 * s[2] * cb, 0.0, 2 * s[2] - 2 * s[0] * cb],
                          [2 * s[0] - 2 * s[1] * cg, 2 * s[1] - 2 * s[0] * cg, 0.0]])
            if abs(np.linalg.det(J)) < 1e-300:
                break
            s = s - np.linalg.solve(J, F)
        if (s <= 0).any():
            continue
        C = s[:, None] * f
        out.append(rigid_from_triads(X, C))
    return out


# --------------------------------------------------------------------------- #
# Lie-algebra coordinates (left-update chart of the pose step)
# --------------------------------------------------------------------------- #
def chart(Rt, Rm, tm):
    """Coordinates (w, v) of the pose (R, t) = Rt about (Rm, tm)."""
    R, t = Rt
    dR = R @ Rm.T
    return np.concatenate([geo.log_so3(dR), t - dR @ tm])


def kernel_inv_diag(pose, prm):
    tn = np.linalg.norm(pose[3:])
    sw, sv = prm["sigma_w"], prm["sigma_t_rel"] * max(tn, 1e-12)
    return 1.0 / np.array([sw, sw, sw, sv, sv, sv]) ** 2


# --------------------------------------------------------------------------- #
# samples of one frame
# --------------------------------------------------------------------------- #
def observations(win, bufs, t, j):
    """Bearing of pixel j's observation in frame t and whether it exists (FP64)."""
    from .gem import Window
    w = Window(win, bufs)
    j = np.atleast_1d(j)
    v, u = np.divmod(j, w.W)
    xt = w.rays(u, v)
    rho = np.asarray(bufs["idepth"], dtype=np.float64).ravel()[j]
    if t == 1:
        ppx, ppy = u.astype(np.float64), v.astype(np.float64)
        zprev = np.ones(j.shape, dtype=bool)
        X = w.flow[0][v, u].astype(np.float64)
        fv = np.isfinite(X).all(-1)
    else:
        R, tt = geo.pose_rt(bufs["pose"][t - 2])
        ppx, ppy, zprev = geo.project(geo.scaled_point(R, tt, xt, rho), *w.intr)
        X, fv = geo.bilinear(w.flow[t - 1], ppx, ppy)
    ox, oy = ppx + X[..., 0], ppy + X[..., 1]
    b = np.stack([(ox - w.intr[2]) / w.intr[0], (oy - w.intr[3]) / w.intr[1], np.ones_like(ox)], -1)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    ok = zprev & fv & np.isfinite(rho) & (rho > 0) & np.isfinite(b).all(-1)
    return b, ok


def draw_triplets(win, bufs, t, it, S, tries):
    """Pixel triplets [S][3] (-1 where a point found no pixel), drawn with probability
    proportional to q_t by rejection (see the module notes)."""
    H, W = win["H"], win["W"]
    npix = H * W
    q = np.asarray(bufs["rigid"], dtype=np.float64)[t - 1].ravel()
    k0, k1 = philox.key_of(win["seed"])
    out = np.full((S, 3), -1, dtype=np.int64)
    g = np.arange(S, dtype=np.uint64)
    for k in range(3):
        pending = np.ones(S, dtype=bool)
        for r in range(tries):
            c1 = np.full(S, k * tries + r, dtype=np.uint64)
            x0, x1, _, _ = philox.philox4x32_10(g, c1, np.full(S, philox.word2(it, t, PURPOSE_POSE), np.uint64),
                                                np.full(S, int(win["window_id"]), np.uint64), k0, k1)
            j = ((x0 * np.uint64(npix)) >> np.uint64(32)).astype(np.int64)
            u = philox.to_unit(x1)
            _, ok = observations(win, bufs, t, j)
            acc = pending & (u < q[j]) & ok
            out[acc, k] = j[acc]
            pending &= ~acc
    return out


def frame_samples(win, bufs, t, it, prm):
    """Pose samples of frame t: for each triplet the P3P solution nearest the current pose
    (6-vectors [S][6]; NaN rows for void samples)."""
    trip = draw_triplets(win, bufs, t, it, prm["samples"], prm["tries"])
    from .gem import Window
    w = Window(win, bufs)
    rho = np.asarray(bufs["idepth"], dtype=np.float64).ravel()
    cur = np.asarray(bufs["pose"][t - 1], dtype=np.float64)
    Rc, tc = geo.pose_rt(cur)
    kinv = kernel_inv_diag(cur, prm)
    out = np.full((len(trip), 6), np.nan)
    for s, jj in enumerate(trip):
        if (jj < 0).any():
            continue
        v, u = np.divmod(jj, w.W)
        Xw = w.rays(u, v) / rho[jj][:, None]
        f, _ = observations(win, bufs, t, jj)
        best, bd = None, np.inf
        for R, tt in p3p(Xw, f):
            d = chart((R, tt), Rc, tc)
            m = float(d @ (kinv * d))
            if np.isfinite(m) and m < bd:
                best, bd = (R, tt), m
        if best is not None:
            out[s] = np.concatenate([geo.log_so3(best[0]), best[1]])
    return out


# --------------------------------------------------------------------------- #
# mode and uncertainty
# --------------------------------------------------------------------------- #
def meanshift(samples, start, kinv, max_steps=100, tol=1e-12):
    """Mode of the Gaussian-kernel mixture of the pose samples [S][6] from `start`: each step
    moves the mode by the kernel-weighted mean of the samples' coordinates about it.
    Returns (mode 6-vector, steps)."""
    samples = samples[np.isfinite(samples).all(1)]
    mode = np.asarray(start, dtype=np.float64).copy()
    Rs = [geo.pose_rt(s) for s in samples]
    for step in range(1, max_steps + 1):
        Rm, tm = geo.pose_rt(mode)
        d = np.array([chart(x, Rm, tm) for x in Rs]).reshape(-1, 6)
        wts = np.exp(-0.5 * (d * d * kinv).sum(1))
        if wts.sum() == 0:
            return mode, step
        delta = (wts[:, None] * d).sum(0) / wts.sum()
        mode = geo.left_update(mode, delta)
        if np.sqrt(float(delta @ (kinv * delta))) < tol:
            return mode, step
    return mode, max_steps


def fit_covariance(samples, mode, kinv, eps, rounds=20):
    """Sigma_t about the mode: 3-sigma inliers of the current fit give the next mean and
    covariance, eigenvalues floored at eps.  Returns (Sigma [6][6], inliers, rounds)."""
    samples = samples[np.isfinite(samples).all(1)]
    Rm, tm = geo.pose_rt(mode)
    d = np.array([chart(geo.pose_rt(s), Rm, tm) for s in samples]).reshape(-1, 6)
    mu = np.zeros(6)
    Sig = np.diag(1.0 / kinv)
    prev = None
    n_in = 0
    for r in range(1, rounds + 1):
        e = d - mu
        m2 = np.einsum("ni,ij,nj->n", e, np.linalg.inv(Sig), e)
        inl = m2 <= 9.0
        if inl.sum() < 7:
            return Sig, n_in, r
        if prev is not None and np.array_equal(inl, prev):
            return Sig, n_in, r
        prev = inl
        n_in = int(inl.sum())
        mu = d[inl].mean(0)
        c = d[inl] - mu
        C = c.T @ c / n_in / KAPPA
        lam, V = np.linalg.eigh(0.5 * (C + C.T))
        Sig = (V * np.maximum(lam, eps)) @ V.T
    return Sig, n_in, rounds


def pose_sample_step(win, bufs, it, prm):
    """The sampled pose M-step over frames t = 1..N in order (each frame's observations use
    the already updated pose of frame t-1).  Updates bufs["pose"]; returns covariances
    [N][36] and info [N][4] = (valid samples, inliers, meanshift steps, fit rounds)."""
    N = win["N"]
    covs = np.zeros((N, 36))
    info = np.zeros((N, 4))
    for t in range(1, N + 1):
        samples = frame_samples(win, bufs, t, it, prm)
        cur = np.asarray(bufs["pose"][t - 1], dtype=np.float64).copy()
        kinv = kernel_inv_diag(cur, prm)
        valid = int(np.isfinite(samples).all(1).sum())
        if valid == 0:
            covs[t - 1] = np.diag(1.0 / kinv).ravel()
            info[t - 1] = (0, 0, 0, 0)
            continue
        mode, steps = meanshift(samples, cur, kinv)
        Sig, n_in, rounds = fit_covariance(samples, mode, kinv, prm["eps"])
        bufs["pose"][t - 1] = mode
        covs[t - 1] = Sig.ravel()
        info[t - 1] = (valid, n_in, steps, rounds)
    return covs, info


DEFAULTS = dict(samples=256, tries=16, sigma_w=0.01, sigma_t_rel=0.02, eps=1e-12)
