"""VOLDOR+ generalized-EM inference over one window, FP64 (test infrastructure).

Model (sec. III-A, Eqs. 1-5): N optical flows X_t (frame t-1 -> t) of a
sliding window, unknown poses T_t, the reference frame's depth and per-frame
rigidness maps W_t; optional depth priors with fixed poses (Eqs. 2-4).  The
state is kept as inverse depth rho = 1/theta.

Rigid flow of reference pixel j at inverse depth rho: p_0 = j,
p_t = pi(T_t, x~_j / rho); the observation for frame t is
o_t = p_{t-1} + X_t(p_{t-1}) (bilinear on frame t-1's grid), the residual is
r_t = |p_t - o_t|.  A term is invalid (uninformative, L1 := L0) when the point
is behind camera t-1 or t, or p_{t-1} falls outside the flow's grid.

One GEM iteration `it` (direction d = it mod 4 of the alternately directed 1D
chains, sec. III-A "Hierarchical Propagation Scheme"):
  coarse level  E-step then M-step on full-length chains of the stride-s lattice;
  local level   E-step then M-step on chains inside T x T tiles at full
                resolution, with the coarse result as an extra candidate;
  pose step     Gauss-Newton on the same MIE energy, frames in order.

Readings of points the paper leaves to the absent VOLDOR reference are listed
in the design notes; the ones that shape code here are named inline.

Buffers (dict of numpy arrays, mirroring the library's buffer struct):
  flow [N][H][W][2], pose [N][6], idepth [H][W], rigid [N][H][W],
  idepth_coarse [Hc][Wc], rigid_coarse [N][Hc][Wc], prior_idepth [P][H][W] (NaN = hole),
  prior_pose [P][6], prior_weight [P][H][W] or None, conf [H][W], stats [8].
"""
import numpy as np

from . import philox, fisk
from . import geometry as geo

SIGMA_FLOOR = 0.005
COARSE, LOCAL = 0, 1
N_SCORE = 29       # energy, H upper triangle (21), g (6), count


# --------------------------------------------------------------------------- #
# levels and chains
# --------------------------------------------------------------------------- #
def lattice_shape(H, W, s):
    """Lattice {(s U + floor(s/2), s V + floor(s/2))} inside the image."""
    o = s // 2
    return (H - o + s - 1) // s, (W - o + s - 1) // s


class Level:
    """Pixel set of one level: level-grid shape and full-resolution coordinates."""

    def __init__(self, win, level):
        H, W = win["H"], win["W"]
        if level == COARSE:
            s = win["coarse_stride"]
            self.h, self.w = lattice_shape(H, W, s)
            V, U = np.mgrid[0:self.h, 0:self.w]
            self.u = (s * U + s // 2).ravel()
            self.v = (s * V + s // 2).ravel()
        else:
            self.h, self.w = H, W
            V, U = np.mgrid[0:H, 0:W]
            self.u, self.v = U.ravel(), V.ravel()
        self.full = self.v * W + self.u


def chains(win, level, d):
    """Alternately directed 1D chains (sec. III-A): groups of equal-length chains, each an
    int array [n, L] of level-grid indices in traversal order.  d = 0 right, 1 down,
    2 left, 3 up.  Coarse level: whole lattice rows / columns; local level: rows /
    columns of T x T tiles (ragged at the image edge)."""
    lv = Level(win, level)
    h, w = lv.h, lv.w
    th, tw = (h, w) if level == COARSE else (win["tile"], win["tile"])
    horizontal, reverse = d % 2 == 0, d >= 2
    groups = {}
    for ty in range(0, h, th):
        for tx in range(0, w, tw):
            y1, x1 = min(ty + th, h), min(tx + tw, w)
            lines = ([y * w + np.arange(tx, x1) for y in range(ty, y1)] if horizontal
                     else [np.arange(ty, y1) * w + x for x in range(tx, x1)])
            for idx in lines:
                groups.setdefault(len(idx), []).append(idx[::-1] if reverse else idx)
    return [np.array(g, dtype=np.int64) for g in groups.values()]


# --------------------------------------------------------------------------- #
# per-pixel likelihood terms
# --------------------------------------------------------------------------- #
class Window:
    def __init__(self, win, bufs):
        self.win, self.b = win, bufs
        self.H, self.W, self.N = win["H"], win["W"], win["N"]
        self.P = int(win.get("P", 0))
        self.intr = (win["fx"], win["fy"], win["cx"], win["cy"])
        self.alpha, self.beta = win["fisk_alpha"], win["fisk_beta"]
        self.L0 = win["outlier_density"]
        self.flow = np.asarray(bufs["flow"], dtype=np.float64)
        self.log_kappa = fisk.prior_log_kappa(win["prior_sigma_rel"], win["prior_uniform_rel"])
        # prior model: 0 Gaussian-uniform mixture on inverse depth (Eq. 3); 1 empirical
        # log-logistic model of the disparity residual (external stereo priors), with
        # prior_sigma_rel its scale (px), prior_fisk_beta its shape, prior_uniform_rel the
        # width (px) of the outlier disparity range and prior_disp_scale = f * baseline
        self.disparity = int(win.get("prior_model", 0)) == 1

    def rays(self, u, v):
        return geo.rays(u, v, *self.intr)

    # -- flows ---------------------------------------------------------------
    def flow_residuals(self, u, v, rho, poses=None):
        """Squared residuals r_t^2 and validity for t = 1..N: arrays [N, *rho.shape]."""
        poses = self.b["pose"] if poses is None else poses
        rho = np.asarray(rho, dtype=np.float64)
        u = np.broadcast_to(np.reshape(u, np.shape(u) + (1,) * (rho.ndim - np.ndim(u))), rho.shape)
        v = np.broadcast_to(np.reshape(v, np.shape(v) + (1,) * (rho.ndim - np.ndim(v))), rho.shape)
        xt = self.rays(u, v)
        px_prev, py_prev = u.astype(np.float64), v.astype(np.float64)
        z_prev = np.ones(rho.shape, dtype=bool)
        r2s, oks = [], []
        for t in range(1, self.N + 1):
            R, tt = geo.pose_rt(poses[t - 1])
            px, py, zok = geo.project(geo.scaled_point(R, tt, xt, rho), *self.intr)
            if t == 1:
                X = self.flow[0][v, u]
                fv = np.isfinite(X).all(-1)
            else:
                X, fv = geo.bilinear(self.flow[t - 1], px_prev, py_prev)
            ok = z_prev & zok & fv
            ex = px - (px_prev + X[..., 0])
            ey = py - (py_prev + X[..., 1])
            r2s.append(np.where(ok, ex * ex + ey * ey, 0.0))
            oks.append(ok)
            px_prev, py_prev, z_prev = px, py, zok
        return np.array(r2s), np.array(oks)

    def flow_costs(self, u, v, rho):
        """Per-frame MIE costs log1p(L0/L1) (log 2 for invalid terms) and validity."""
        r2, ok = self.flow_residuals(u, v, rho)
        cost = np.where(ok, fisk.flow_term(self._floor_r2(r2), self.alpha, self.beta, self.L0), fisk.LOG2)
        return cost, ok

    def emissions(self, u, v, rho):
        """HMM emissions (L0, L1) per frame, true densities in px^-2; invalid -> (L0, L0)."""
        r2, ok = self.flow_residuals(u, v, rho)
        L1 = fisk.planar_density(np.sqrt(self._floor_r2(r2)), self.alpha, self.beta)
        return np.full(r2.shape, self.L0), np.where(ok, L1, self.L0), ok

    def _floor_r2(self, r2):
        # for shape < 2 the planar density diverges at r = 0; floor r at 1e-3 alpha
        return r2 if self.beta >= 2.0 else np.maximum(r2, (1e-3 * self.alpha) ** 2)

    # -- depth priors (Eqs. 3-4) -----------------------------------------------
    def prior_z(self, k, u, v, rho):
        """Normalised inverse-depth difference z = (rho^(l) - 1/phi_z) / sigma for prior k,
        with l the nearest pixel of the transfer of the candidate into prior camera k.
        Reading of the garbled l = pi(theta_2^j, T^_k): theta_2 is the candidate depth.
        With the empirical disparity model (prior_model 1) z is the signed disparity
        residual fb (rho^(l) - 1/phi_z) instead."""
        rho = np.asarray(rho, dtype=np.float64)
        u = np.broadcast_to(np.reshape(u, np.shape(u) + (1,) * (rho.ndim - np.ndim(u))), rho.shape)
        v = np.broadcast_to(np.reshape(v, np.shape(v) + (1,) * (rho.ndim - np.ndim(v))), rho.shape)
        R, t = geo.pose_rt(self.b["prior_pose"][k])
        Q = geo.scaled_point(R, t, self.rays(u, v), rho)       # rho * (R X + t)
        lx, ly, zok = geo.project(Q, *self.intr)
        lx = np.floor(lx + 0.5)
        ly = np.floor(ly + 0.5)
        inside = zok & (lx >= 0) & (lx <= self.W - 1) & (ly >= 0) & (ly <= self.H - 1)
        lxi = np.where(inside, lx, 0).astype(np.int64)
        lyi = np.where(inside, ly, 0).astype(np.int64)
        rh = np.asarray(self.b["prior_idepth"][k], dtype=np.float64)[lyi, lxi]
        ok = inside & np.isfinite(rh) & (rh > 0)
        rh = np.where(ok, rh, 1.0)
        inv_phi = rho / np.where(zok, Q[..., 2], 1.0)           # 1 / phi_z = rho / (rho Q_z)
        if self.disparity:
            z = fisk.disparity_residual(rh, inv_phi, self.win["prior_disp_scale"])
        else:
            z = (rh - inv_phi) / (self.win["prior_sigma_rel"] * rh)
        return np.where(ok, z, 0.0), ok

    def prior_cost(self, z):
        """MIE cost of a prior term with a valid transfer (Eq. 4 on Eq. 3's mixture, or on the
        empirical disparity model)."""
        if self.disparity:
            w = self.win
            return fisk.disparity_prior_term(z, w["prior_sigma_rel"], w["prior_fisk_beta"], w["prior_uniform_rel"])
        return fisk.prior_term(z, self.log_kappa)

    def prior_q(self, z, pi_hat):
        if self.disparity:
            w = self.win
            return fisk.disparity_prior_posterior(z, w["prior_sigma_rel"], w["prior_fisk_beta"],
                                                  w["prior_uniform_rel"], pi_hat)
        return fisk.prior_posterior(z, self.log_kappa, pi_hat)

    def prior_weight(self, k, u, v):
        pw = self.b.get("prior_weight")
        if pw is None:
            return np.full(np.shape(u), float(self.win["prior_inlier_default"]))
        return np.asarray(pw[k], dtype=np.float64)[v, u]

    def prior_posteriors(self, u, v, rho):
        """q^_k at the given (current) inverse depth: [P, n]; 0 where there is no term."""
        out = np.zeros((self.P,) + np.shape(u))
        for k in range(self.P):
            z, ok = self.prior_z(k, u, v, rho)
            out[k] = np.where(ok, self.prior_q(z, self.prior_weight(k, u, v)), 0.0)
        return out

    # -- total per-pixel energy (Eq. 5) ---------------------------------------
    def energy(self, u, v, rho, q, qhat):
        """E_j(rho) = sum_t q_t log1p(L0/L1_t) + sum_k q^_k softplus(log kappa + z_k^2/2)
        for pixels (u, v) [n], candidates rho [n, K], q [N, n], qhat [P, n] -> [n, K].
        A prior term with q^ = 0 is absent; one whose candidate transfer is invalid is
        uninformative (q^ log 2)."""
        cost, _ = self.flow_costs(u, v, rho)
        E = np.einsum("tn,tnk->nk", q, cost)
        for k in range(self.P):
            z, ok = self.prior_z(k, u, v, rho)
            term = np.where(ok, self.prior_cost(z), fisk.LOG2)
            E = E + np.where(qhat[k][:, None] > 0, qhat[k][:, None] * term, 0.0)
        return E


# --------------------------------------------------------------------------- #
# E-step: rigidness forward-backward (sec. III-A; HMM smoothing on 1D chains)
# --------------------------------------------------------------------------- #
def forward_backward(e0, e1, gamma):
    """Two-state HMM on chains: emissions e0, e1 [n, L] (state 1 = rigid / inlier),
    initial (1/2, 1/2), symmetric transition gamma.  Scaled forward and backward
    recursions; returns q = P(W_i = 1 | chain) [n, L] and log Z [n] = sum of log scales."""
    n, L = e0.shape
    a = np.zeros((n, L, 2))
    x0, x1 = 0.5 * e0[:, 0], 0.5 * e1[:, 0]
    c = x0 + x1
    a[:, 0, 0], a[:, 0, 1] = x0 / c, x1 / c
    logz = np.log(c)
    for i in range(1, L):
        p0 = gamma * a[:, i - 1, 0] + (1 - gamma) * a[:, i - 1, 1]
        p1 = (1 - gamma) * a[:, i - 1, 0] + gamma * a[:, i - 1, 1]
        x0, x1 = p0 * e0[:, i], p1 * e1[:, i]
        c = x0 + x1
        a[:, i, 0], a[:, i, 1] = x0 / c, x1 / c
        logz = logz + np.log(c)
    b = np.zeros((n, L, 2))
    b[:, L - 1] = 0.5
    for i in range(L - 2, -1, -1):
        m0, m1 = e0[:, i + 1] * b[:, i + 1, 0], e1[:, i + 1] * b[:, i + 1, 1]
        y0 = gamma * m0 + (1 - gamma) * m1
        y1 = (1 - gamma) * m0 + gamma * m1
        s = y0 + y1
        b[:, i, 0], b[:, i, 1] = y0 / s, y1 / s
    num = a[:, :, 1] * b[:, :, 1]
    q = num / (a[:, :, 0] * b[:, :, 0] + num)
    return q, logz


def rigidness_fb(win, bufs, it, level, select=None):
    """E-step of one level at the current inverse depth and poses.  Writes the rigidness
    posteriors of that level's pixels (rigid, or rigid_coarse for the coarse level) and
    returns sum of log Z over chains and frames.

    chain_axis 0 (paper): per frame, chains are the level's 1D chains in direction it mod 4.
    chain_axis 1: per pixel, the chain runs over the frame window t = 1..N.
    `select(groups) -> groups` may restrict the chains evaluated (sampled checks)."""
    w = Window(win, bufs)
    lv = Level(win, level)
    gamma = win["hmm_gamma"]
    rho = np.asarray(bufs["idepth"], dtype=np.float64).ravel()[lv.full]
    out = bufs["rigid_coarse" if level == COARSE else "rigid"].reshape(w.N, -1)
    loglik = 0.0
    if win.get("chain_axis", 0) == 1:
        e0, e1, _ = w.emissions(lv.u, lv.v, rho)                    # [N, n]
        q, logz = forward_backward(e0.T, e1.T, gamma)
        out[:, :] = q.T
        return float(logz.sum())
    groups = chains(win, level, it % 4)
    if select is not None:
        groups = select(groups)
    for g in groups:
        flat = g.ravel()
        e0, e1, _ = w.emissions(lv.u[flat], lv.v[flat], rho[flat])  # [N, n*L]
        for t in range(w.N):
            q, logz = forward_backward(e0[t].reshape(g.shape), e1[t].reshape(g.shape), gamma)
            out[t, flat] = q.ravel()
            loglik += float(logz.sum())
    return loglik


# --------------------------------------------------------------------------- #
# M-step: candidate sampling and propagation (sec. III-A, Eq. 5)
# --------------------------------------------------------------------------- #
def perturb_sigma(win, it):
    """Relative perturbation width: sigma0 halved every two iterations, floored."""
    return max(win["perturb_sigma0"] * 2.0 ** (-(it // 2)), SIGMA_FLOOR)


def candidates_random(win, lv, it, level, rho_cur, pix):
    """Slots 3..K-1 for level pixels `pix` (level-grid indices): even slots uniform over
    [rho_min, rho_max], odd slots a relative perturbation of the current value."""
    K = win["n_candidates"]
    lo, hi = win["idepth_min"], win["idepth_max"]
    sig = perturb_sigma(win, it)
    G = (K - 3 + 3) // 4
    out = np.zeros((len(pix), max(K - 3, 0)))
    if G == 0:
        return out
    U = np.concatenate([philox.uniforms(pix, g, it, level, philox.PURPOSE_CAND, win["window_id"],
                                        win["seed"]) for g in range(G)], axis=-1)
    for k in range(3, K):
        uk = U[:, k - 3]
        out[:, k - 3] = (lo + uk * (hi - lo)) if k % 2 == 0 else \
            np.clip(rho_cur * (1.0 + sig * (2.0 * uk - 1.0)), lo, hi)
    return out


def depth_update(win, bufs, it, level, select=None):
    """M-step of one level.  Each chain is swept in direction it mod 4; pixel i takes the
    argmin of E_j over the slots
      0 current value, 1 the predecessor's updated value (pixel 0: its own current value),
      2 the coarse result at the pixel's lattice cell (local level only),
      3..K-1 Philox draws,
    with ties to the lowest slot.  The rigidness posteriors of the level's last E-step
    and the prior posteriors at the current value stay fixed during the sweep.
    Writes idepth_coarse (coarse level) or idepth (local level)."""
    w = Window(win, bufs)
    lv = Level(win, level)
    K = win["n_candidates"]
    rho_full = np.asarray(bufs["idepth"], dtype=np.float64).ravel()
    rho_cur = rho_full[lv.full].copy()
    if level == COARSE:
        q = np.asarray(bufs["rigid_coarse"], dtype=np.float64).reshape(w.N, -1)
        out = bufs["idepth_coarse"].reshape(-1)
        rc = None
    else:
        q = np.asarray(bufs["rigid"], dtype=np.float64).reshape(w.N, -1)
        out = bufs["idepth"].reshape(-1)
        s = win["coarse_stride"]
        hc, wc = lattice_shape(w.H, w.W, s)
        U = np.minimum(lv.u // s, wc - 1)
        V = np.minimum(lv.v // s, hc - 1)
        rc = np.asarray(bufs["idepth_coarse"], dtype=np.float64)[V, U]
    groups = chains(win, level, it % 4)
    if select is not None:
        groups = select(groups)
    for g in groups:
        n, L = g.shape
        qhat = w.prior_posteriors(lv.u[g.ravel()], lv.v[g.ravel()], rho_cur[g.ravel()]).reshape(w.P, n, L)
        rand = candidates_random(win, lv, it, level, rho_cur[g.ravel()], g.ravel()).reshape(n, L, -1)
        prev = None
        for i in range(L):
            pix = g[:, i]
            cand = np.zeros((n, K))
            cand[:, 0] = rho_cur[pix]
            cand[:, 1] = rho_cur[pix] if i == 0 else prev
            cand[:, 2] = rc[pix] if rc is not None else rho_cur[pix]
            cand[:, 3:] = rand[:, i]
            E = w.energy(lv.u[pix], lv.v[pix], cand, q[:, pix], qhat[:, :, i])
            if rc is None:
                E[:, 2] = np.inf
            best = np.argmin(E, axis=1)                 # first minimum: lowest slot wins ties
            prev = cand[np.arange(n), best]
            out[pix] = prev
    return out


# --------------------------------------------------------------------------- #
# pose step (reading: Gauss-Newton on the same MIE energy; see design notes)
# --------------------------------------------------------------------------- #
def _jac_rows(Q, rho, fx, fy):
    """d p / d delta for a left pose update, p = pi(Q), Q = rho (R X + t):
    dQ/d(dw, dv) = [-[Q]x | rho I];  dp/dQ = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]."""
    x, y, z = Q[..., 0], Q[..., 1], Q[..., 2]
    z = np.where(z > 0, z, 1.0)
    dp = np.zeros(Q.shape[:-1] + (2, 3))
    dp[..., 0, 0] = fx / z
    dp[..., 0, 2] = -fx * x / (z * z)
    dp[..., 1, 1] = fy / z
    dp[..., 1, 2] = -fy * y / (z * z)
    M = np.zeros(Q.shape[:-1] + (3, 6))
    qx, qy, qz = Q[..., 0], Q[..., 1], Q[..., 2]
    M[..., 0, 1], M[..., 0, 2] = qz, -qy          # -[Q]x
    M[..., 1, 0], M[..., 1, 2] = -qz, qx
    M[..., 2, 0], M[..., 2, 1] = qy, -qx
    M[..., 0, 3] = M[..., 1, 4] = M[..., 2, 5] = rho
    return dp @ M


def pose_score(win, bufs, t, cand):
    """Score candidate poses for frame t (1..N): for each candidate the MIE energy
    sum_j q_t^j cost_t^j, the IRLS normal equations H = sum w J^T J, g = sum w J^T e of
    the residual e = p_t - o_t with w = q d cost / d(r^2), and the number of valid terms.
    o_t uses the current pose of frame t-1.  Returns [n_cand, 29]:
    energy, H upper triangle row-major (21), g (6), count.

    Reading of the pose step's term set: a term counts only where the reprojection p_t lies
    inside frame t's image (a flow end point is observed nowhere else); otherwise it is
    invalid like any other (cost q log 2, no weight).  Without this, points that pass just
    in front of camera t (Q_z -> 0+) enter with weight ~ 1/Q_z^2 and decide the step."""
    w = Window(win, bufs)
    cand = np.atleast_2d(np.asarray(cand, dtype=np.float64))
    V, U = np.mgrid[0:w.H, 0:w.W]
    u, v = U.ravel(), V.ravel()
    rho = np.asarray(bufs["idepth"], dtype=np.float64).ravel()
    q = np.asarray(bufs["rigid"], dtype=np.float64)[t - 1].ravel()
    xt = w.rays(u, v)
    if t == 1:
        ppx, ppy = u.astype(np.float64), v.astype(np.float64)
        zprev = np.ones(u.shape, dtype=bool)
        X = w.flow[0][v, u]
        fv = np.isfinite(X).all(-1)
    else:
        R, tt = geo.pose_rt(bufs["pose"][t - 2])
        ppx, ppy, zprev = geo.project(geo.scaled_point(R, tt, xt, rho), *w.intr)
        X, fv = geo.bilinear(w.flow[t - 1], ppx, ppy)
    ox, oy = ppx + X[:, 0], ppy + X[:, 1]
    iu = np.triu_indices(6)
    out = np.zeros((len(cand), N_SCORE))
    for c, pc in enumerate(cand):
        R, tt = geo.pose_rt(pc)
        Q = geo.scaled_point(R, tt, xt, rho)
        px, py, zok = geo.project(Q, *w.intr)
        inside = (px >= 0) & (px <= w.W - 1) & (py >= 0) & (py <= w.H - 1)
        ok = zprev & zok & fv & inside
        e = np.stack([px - ox, py - oy], -1)
        r2 = np.where(ok, (e * e).sum(-1), 0.0)
        r2f = w._floor_r2(r2)
        cost = np.where(ok, fisk.flow_term(r2f, w.alpha, w.beta, w.L0), fisk.LOG2)
        wt = np.where(ok, q * fisk.flow_weight(r2f, w.alpha, w.beta, w.L0), 0.0)
        J = _jac_rows(Q, rho, w.intr[0], w.intr[1])              # [n, 2, 6]
        J = np.where(ok[:, None, None], J, 0.0)
        e = np.where(ok[:, None], e, 0.0)
        H = np.einsum("n,nai,naj->ij", wt, J, J)
        g = np.einsum("n,nai,na->i", wt, J, e)
        out[c, 0] = float((q * cost).sum())
        out[c, 1:22] = H[iu]
        out[c, 22:28] = g
        out[c, 28] = float(ok.sum())
    return out


def unpack_normal_equations(row):
    H = np.zeros((6, 6))
    H[np.triu_indices(6)] = row[1:22]
    H = H + np.triu(H, 1).T
    return H, np.asarray(row[22:28], dtype=np.float64)


PIVOT_REL = 1e-12


def cholesky_solve(A, b):
    """Solve A x = b for symmetric positive definite A by Cholesky A = L L^T, plain loops.
    Returns None when a pivot is not finite or not above 1e-12 times the largest diagonal
    entry of A (numerically singular)."""
    n = len(b)
    tol = PIVOT_REL * max(float(np.max(np.diag(A))), 0.0)
    L = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            s = A[i, j] - sum(L[i, k] * L[j, k] for k in range(j))
            if i == j:
                if not (np.isfinite(s) and s > tol):
                    return None
                L[i, i] = np.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (b[i] - sum(L[i, k] * y[k] for k in range(i))) / L[i, i]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - sum(L[k, i] * x[k] for k in range(i + 1, n))) / L[i, i]
    return x


def pose_solve_step(row):
    """GN increment from a score row: (H + 1e-9 tr(H)/6 I) delta = -g; None if not PD."""
    H, g = unpack_normal_equations(row)
    lam = 1e-9 * np.trace(H) / 6.0
    return cholesky_solve(H + lam * np.eye(6), -g)


def pose_step(win, bufs, it=0):
    """Frames t = 1..N in order, pose_gn_steps Gauss-Newton steps each (frame t-1's pose is
    already updated when frame t is scored).  A singular system leaves the pose unchanged."""
    for t in range(1, win["N"] + 1):
        for _ in range(win["pose_gn_steps"]):
            row = pose_score(win, bufs, t, bufs["pose"][t - 1][None])[0]
            delta = pose_solve_step(row)
            if delta is None:
                break
            bufs["pose"][t - 1] = geo.left_update(bufs["pose"][t - 1], delta)


# --------------------------------------------------------------------------- #
# init, iteration, confidence (Eq. 6)
# --------------------------------------------------------------------------- #
def prior_bootstrap(win, bufs, rounds=2):
    """Inverse depth of every reference pixel read off the first depth prior (sec. III-A:
    VOLDOR+ starts from explicit priors where VOLDOR bootstraps its hidden variables
    deterministically).  The value sought makes the transfer into prior 0's camera meet the
    prior at the pixel it lands on: with X = x~ / rho, R X + t has depth a / rho + t_z
    (a = r_3 . x~), so 1 / phi_z = rho^(l) solves to rho = rho^(l) a / (1 - rho^(l) t_z).
    l depends on rho; two fixed-point rounds start from the prior's value at the same pixel
    (for an identity prior pose the first round is exact).  Returns (rho, ok); ok is false
    where a round lands outside the image or behind the camera, or meets a hole (NaN or
    non-positive value) or a non-positive solution."""
    H, W = win["H"], win["W"]
    fx, fy, cx, cy = win["fx"], win["fy"], win["cx"], win["cy"]
    V, U = np.mgrid[0:H, 0:W]
    x = geo.rays(U, V, fx, fy, cx, cy)
    R, t = geo.pose_rt(bufs["prior_pose"][0])
    pri = np.asarray(bufs["prior_idepth"][0], dtype=np.float64)
    a = x @ R[2]
    rho = pri.copy()
    ok = np.isfinite(rho) & (rho > 0)
    for _ in range(rounds):
        Q = x @ R.T / np.where(ok, rho, 1.0)[..., None] + t
        lx, ly, zok = geo.project(Q, fx, fy, cx, cy)
        lx = np.floor(lx + 0.5)
        ly = np.floor(ly + 0.5)
        ok &= zok & (lx >= 0) & (lx <= W - 1) & (ly >= 0) & (ly <= H - 1)
        rh = pri[np.where(ok, ly, 0).astype(np.int64), np.where(ok, lx, 0).astype(np.int64)]
        den = 1.0 - rh * t[2]
        ok &= np.isfinite(rh) & (rh > 0) & (den > 0) & (a > 0)
        rho = np.where(ok, rh * a / np.where(ok, den, 1.0), 0.0)
    return rho, ok


def init_idepth(win, bufs):
    """Initial inverse depth.  Random rho_min + u (rho_max - rho_min), u from Philox (pixel
    index, group 0, iteration 0, local level, purpose INIT), first word; with a depth prior
    (P >= 1, unless init_random is set) every pixel that prior_bootstrap resolves starts at
    that value instead, clamped to [rho_min, rho_max]."""
    H, W = win["H"], win["W"]
    u = philox.uniforms(np.arange(H * W), 0, 0, LOCAL, philox.PURPOSE_INIT, win["window_id"],
                        win["seed"])[:, 0]
    lo, hi = win["idepth_min"], win["idepth_max"]
    rho = (lo + u * (hi - lo)).reshape(H, W)
    if win.get("P", 0) >= 1 and not win.get("init_random", 0) and bufs.get("prior_idepth") is not None:
        boot, ok = prior_bootstrap(win, bufs)
        rho = np.where(ok, np.clip(boot, lo, hi), rho)
    bufs["idepth"][...] = rho


def gem_step(win, bufs, it):
    """One GEM iteration: coarse E, coarse M, local E, local M, pose step."""
    rigidness_fb(win, bufs, it, COARSE)
    depth_update(win, bufs, it, COARSE)
    rigidness_fb(win, bufs, it, LOCAL)
    depth_update(win, bufs, it, LOCAL)
    pose_step(win, bufs, it)


def finalize(win, bufs, it):
    """Final local E-step (direction it mod 4), confidence map and statistics.

    C^j = (sum_t q_t^j + sum_k q^_k^j) / (N + P)   (Eq. 6; holes count with q^ = 0).
    stats: [0] log-likelihood sum of log Z, [1] MIE energy sum_j E_j(rho_j),
           [2] valid flow terms, [3] invalid flow terms, [4] prior terms with a valid
           transfer (not a hole) at the final depth,
           [5] sum of C, [6], [7] zero."""
    w = Window(win, bufs)
    loglik = rigidness_fb(win, bufs, it, LOCAL)
    lv = Level(win, LOCAL)
    rho = np.asarray(bufs["idepth"], dtype=np.float64).ravel()
    q = np.asarray(bufs["rigid"], dtype=np.float64).reshape(w.N, -1)
    qhat = w.prior_posteriors(lv.u, lv.v, rho)
    conf = (q.sum(0) + qhat.sum(0)) / (w.N + w.P)
    bufs["conf"][...] = conf.reshape(w.H, w.W)
    E = w.energy(lv.u, lv.v, rho[:, None], q, qhat)[:, 0]
    _, ok = w.flow_costs(lv.u, lv.v, rho)
    stats = np.zeros(8)
    stats[0] = loglik
    stats[1] = E.sum()
    stats[2] = ok.sum()
    stats[3] = ok.size - ok.sum()
    stats[4] = sum(int(w.prior_z(k, lv.u, lv.v, rho)[1].sum()) for k in range(w.P))
    stats[5] = conf.sum()
    bufs["stats"][...] = stats
    return stats


def alloc_buffers(win, flow, pose, prior_idepth=None, prior_pose=None, prior_weight=None):
    """FP64 buffer set for one window (copies of the inputs)."""
    H, W, N = win["H"], win["W"], win["N"]
    hc, wc = lattice_shape(H, W, win["coarse_stride"])
    P = int(win.get("P", 0))
    return dict(
        flow=np.asarray(flow, dtype=np.float32).copy(),
        pose=np.asarray(pose, dtype=np.float64).copy(),
        idepth=np.zeros((H, W)), rigid=np.zeros((N, H, W)),
        idepth_coarse=np.zeros((hc, wc)), rigid_coarse=np.zeros((N, hc, wc)),
        prior_idepth=(np.asarray(prior_idepth, dtype=np.float64).copy() if P else np.zeros((0, H, W))),
        prior_pose=(np.asarray(prior_pose, dtype=np.float64).copy() if P else np.zeros((0, 6))),
        prior_weight=(None if prior_weight is None else np.asarray(prior_weight, dtype=np.float64).copy()),
        conf=np.zeros((H, W)), stats=np.zeros(8))


def run(win, bufs, iters=None, init=True):
    """Plain GEM from random initial depth: init, iterations 0..I-1, finalize."""
    iters = win.get("iters", 5) if iters is None else iters
    if init:
        init_idepth(win, bufs)
    for it in range(iters):
        gem_step(win, bufs, it)
    return finalize(win, bufs, iters - 1)
