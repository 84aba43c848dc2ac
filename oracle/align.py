"""Robust point-to-plane inverse-depth keyframe alignment, FP64 (test infrastructure).

Sec. III-B "Keyframe Alignment", Eq. 10 with the criterion of Eq. 12 (no
photometric term, s = 1 for absolutely scaled depth):

  E_geo = sum_j C^j psi( <n(l), P1(l) - Q_j> / (s theta1(l) Q_j,z) ),
  Q_j = T X2_j (map-2 point j moved into camera 1), l = pixel of its projection,

written in inverse depth as r_j = rho1(l) <n(l), P1(l) - Q_j> / (s Q_j,z).
Readings: l is the nearest pixel, held fixed within a Gauss-Newton step;
normals come from central differences of map 1 with a depth-discontinuity
test; psi is Huber (scale delta) or Cauchy; C^j is map 2's confidence;
undamped Gauss-Newton; the covariance is H^-1 of the weighted system at the
final pose (Eq. 12's (J^T J)^-1 with the robust weights).
"""
import numpy as np

from . import geometry as geo
from .gem import cholesky_solve

HUBER, CAUCHY = 0, 1
ESINGULAR = 4


def normals(rho1, fx, fy, cx, cy, disc_rel):
    """Unit normals of map 1: n = normalise((P(l+x) - P(l-x)) x (P(l+y) - P(l-y))), turned
    to face the camera (n . P < 0).  Invalid on the border, where a neighbour is missing
    or non-positive, or where |rho_nb - rho_l| > disc_rel * rho_l."""
    rho1 = np.asarray(rho1, dtype=np.float64)
    H, W = rho1.shape
    V, U = np.mgrid[0:H, 0:W]
    ok0 = np.isfinite(rho1) & (rho1 > 0)
    r = np.where(ok0, rho1, 1.0)
    P = geo.rays(U, V, fx, fy, cx, cy) / r[..., None]
    n = np.zeros((H, W, 3))
    valid = np.zeros((H, W), dtype=bool)
    c = (slice(1, H - 1), slice(1, W - 1))
    nb = [(slice(1, H - 1), slice(2, W)), (slice(1, H - 1), slice(0, W - 2)),
          (slice(2, H), slice(1, W - 1)), (slice(0, H - 2), slice(1, W - 1))]
    ok = ok0[c].copy()
    for s in nb:
        ok &= ok0[s] & (np.abs(np.where(ok0[s], rho1[s], np.inf) - r[c]) <= disc_rel * r[c])
    dx = P[nb[0]] - P[nb[1]]
    dy = P[nb[2]] - P[nb[3]]
    cr = np.cross(dx, dy)
    ln = np.linalg.norm(cr, axis=-1)
    ok &= ln > 0
    cr = cr / np.where(ln > 0, ln, 1.0)[..., None]
    flip = (cr * P[c]).sum(-1) > 0
    cr[flip] *= -1
    n[c] = cr
    valid[c] = ok
    return n, valid


def robust(r, kind, scale):
    """psi(r) and the IRLS weight psi'(r)/r."""
    a = np.abs(r)
    if kind == HUBER:
        psi = np.where(a <= scale, 0.5 * r * r, scale * (a - 0.5 * scale))
        w = np.where(a <= scale, 1.0, scale / np.where(a > 0, a, 1.0))
    else:
        psi = 0.5 * scale * scale * np.log1p((r / scale) ** 2)
        w = 1.0 / (1.0 + (r / scale) ** 2)
    return psi, w


def linearize(ap, rho1, nrm, nvalid, rho2, conf2, pose, terms=False):
    """Residuals, Jacobians and weights of every valid map-2 pixel at `pose`
    (T: camera 2 -> camera 1).  Returns H (6x6), g (6), cost, count
    (and, with terms=True, the per-pixel residual, Jacobian and validity too)."""
    fx, fy, cx, cy = ap["fx"], ap["fy"], ap["cx"], ap["cy"]
    s = ap["scale_s"]
    H_, W_ = rho1.shape
    V, U = np.mgrid[0:H_, 0:W_]
    rho2 = np.asarray(rho2, dtype=np.float64)
    c2 = np.asarray(conf2, dtype=np.float64)
    ok = np.isfinite(rho2) & (rho2 > 0) & np.isfinite(c2)
    r2s = np.where(ok, rho2, 1.0)
    X2 = geo.rays(U, V, fx, fy, cx, cy) / r2s[..., None]
    R, t = geo.pose_rt(pose)
    Q = X2 @ R.T + t
    Qz = Q[..., 2]
    ok &= Qz > 0
    Qzs = np.where(ok, Qz, 1.0)
    lx = np.floor(fx * Q[..., 0] / Qzs + cx + 0.5)
    ly = np.floor(fy * Q[..., 1] / Qzs + cy + 0.5)
    ok &= (lx >= 1) & (lx <= W_ - 2) & (ly >= 1) & (ly <= H_ - 2)
    li = np.where(ok, lx, 1).astype(np.int64)
    lj = np.where(ok, ly, 1).astype(np.int64)
    ok &= nvalid[lj, li]
    n = nrm[lj, li]
    r1 = np.asarray(rho1, dtype=np.float64)[lj, li]
    r1 = np.where(ok, r1, 1.0)
    P1 = geo.rays(li, lj, fx, fy, cx, cy) / r1[..., None]
    r = r1 * (n * (P1 - Q)).sum(-1) / (s * Qzs)
    # dr/dQ = -(1/Qz) (rho1 n / s + r e_z);  dQ/d(dw, dv) = [-[Q]x | I]
    drdQ = -(r1[..., None] * n / s) / Qzs[..., None]
    drdQ[..., 2] -= r / Qzs
    qx, qy, qz = Q[..., 0], Q[..., 1], Q[..., 2]
    J = np.zeros(Q.shape[:-1] + (6,))
    # row vector a times -[Q]x = (a1 (-qz) + a2 qy, a0 qz - a2 qx, -a0 qy + a1 qx)
    a0, a1, a2 = drdQ[..., 0], drdQ[..., 1], drdQ[..., 2]
    J[..., 0] = -a1 * qz + a2 * qy
    J[..., 1] = a0 * qz - a2 * qx
    J[..., 2] = -a0 * qy + a1 * qx
    J[..., 3:] = drdQ
    psi, w = robust(np.where(ok, r, 0.0), ap["robust"], ap["robust_scale"])
    Wt = np.where(ok, c2 * w, 0.0)
    Jv = np.where(ok[..., None], J, 0.0)
    rv = np.where(ok, r, 0.0)
    Hm = np.einsum("n,ni,nj->ij", Wt.ravel(), Jv.reshape(-1, 6), Jv.reshape(-1, 6))
    g = np.einsum("n,ni,n->i", Wt.ravel(), Jv.reshape(-1, 6), rv.ravel())
    cost = float(np.where(ok, c2 * psi, 0.0).sum())
    if terms:
        return Hm, g, cost, int(ok.sum()), rv, Jv, ok
    return Hm, g, cost, int(ok.sum())


def align_pair(ap, rho1, rho2, conf2, pose0):
    """Gauss-Newton from pose0 for ap['gn_steps'] steps; then H at the final pose gives the
    covariance.  Returns (pose, cov [6x6], stats [cost0, cost_final, count_final, steps], status)."""
    nrm, nvalid = normals(rho1, ap["fx"], ap["fy"], ap["cx"], ap["cy"], ap["normal_disc_rel"])
    pose = np.asarray(pose0, dtype=np.float64).copy()
    status = 0
    cost0 = None
    steps = 0
    for _ in range(ap["gn_steps"]):
        Hm, g, cost, cnt = linearize(ap, rho1, nrm, nvalid, rho2, conf2, pose)
        if cost0 is None:
            cost0 = cost
        delta = cholesky_solve(Hm, -g)
        if delta is None:
            status = ESINGULAR
            break
        pose = geo.left_update(pose, delta)
        steps += 1
    Hm, g, cost, cnt = linearize(ap, rho1, nrm, nvalid, rho2, conf2, pose)
    if cost0 is None:
        cost0 = cost
    cov = np.full((6, 6), np.nan)
    if status == 0:
        cols = [cholesky_solve(Hm, e) for e in np.eye(6)]
        if any(c is None for c in cols):
            status = ESINGULAR
        else:
            cov = np.array(cols).T
    return pose, cov, np.array([cost0, cost, cnt, steps], dtype=np.float64), status


def align_p2p(ap, idepth1, idepth2, conf2, pose_inout):
    """All pairs: updates pose_inout [n][6]; returns cov [n][36], stats [n][4], status [n]."""
    n = len(idepth1)
    cov = np.zeros((n, 36))
    stats = np.zeros((n, 4))
    status = np.zeros(n, dtype=np.int32)
    for i in range(n):
        p, c, s, st = align_pair(ap, idepth1[i], idepth2[i], conf2[i], pose_inout[i])
        pose_inout[i] = p          # on ESINGULAR: completed steps kept, the failing one not applied
        cov[i] = c.ravel()
        stats[i] = s
        status[i] = st
    return cov, stats, status


# --------------------------------------------------------------------------- #
# 7-DoF alignment: relative motion and scale, Levenberg-Marquardt
# --------------------------------------------------------------------------- #
LM_LAMBDA0 = 1e-4
LM_LAMBDA_MIN, LM_LAMBDA_MAX = 1e-12, 1e12


def linearize_sim3(ap, rho1, nrm, nvalid, rho2, conf2, pose, s):
    """Eq. 10 with both the motion T (camera 2 -> camera 1) and the relative depth scale s
    unknown (sec. III-B: "we estimate both their relative motion T and scale factor s").
    Reading: map 1's geometry is scaled by s, so the plane of pixel l passes through s P1(l):
      r = rho1 <n, s P1 - Q> / (s Q_z),
    which reduces to Eq. 9's 1/(s theta1) - 1/phi_z for a fronto-parallel plane.  The
    unknowns are updated by the left pose update and s <- s exp(d sigma).
    Returns H (7x7), g (7), cost, count."""
    Hm6, g6, cost, cnt, r, J6, ok = _sim3_terms(ap, rho1, nrm, nvalid, rho2, conf2, pose, s)
    return Hm6, g6, cost, cnt


def _sim3_terms(ap, rho1, nrm, nvalid, rho2, conf2, pose, s):
    fx, fy, cx, cy = ap["fx"], ap["fy"], ap["cx"], ap["cy"]
    H_, W_ = rho1.shape
    V, U = np.mgrid[0:H_, 0:W_]
    rho2 = np.asarray(rho2, dtype=np.float64)
    c2 = np.asarray(conf2, dtype=np.float64)
    ok = np.isfinite(rho2) & (rho2 > 0) & np.isfinite(c2)
    r2s = np.where(ok, rho2, 1.0)
    X2 = geo.rays(U, V, fx, fy, cx, cy) / r2s[..., None]
    R, t = geo.pose_rt(pose)
    Q = X2 @ R.T + t
    Qz = Q[..., 2]
    ok &= Qz > 0
    Qzs = np.where(ok, Qz, 1.0)
    lx = np.floor(fx * Q[..., 0] / Qzs + cx + 0.5)
    ly = np.floor(fy * Q[..., 1] / Qzs + cy + 0.5)
    ok &= (lx >= 1) & (lx <= W_ - 2) & (ly >= 1) & (ly <= H_ - 2)
    li = np.where(ok, lx, 1).astype(np.int64)
    lj = np.where(ok, ly, 1).astype(np.int64)
    ok &= nvalid[lj, li]
    n = nrm[lj, li]
    r1 = np.where(ok, np.asarray(rho1, dtype=np.float64)[lj, li], 1.0)
    P1 = geo.rays(li, lj, fx, fy, cx, cy) / r1[..., None]
    nQ = (n * Q).sum(-1)
    r = r1 * ((n * P1).sum(-1) * s - nQ) / (s * Qzs)
    # dr/dQ = -(1/Qz) (rho1 n / s + r e_z);  dr/dsigma = s dr/ds = rho1 <n, Q> / (s Qz)
    drdQ = -(r1[..., None] * n / s) / Qzs[..., None]
    drdQ[..., 2] -= r / Qzs
    qx, qy, qz = Q[..., 0], Q[..., 1], Q[..., 2]
    J = np.zeros(Q.shape[:-1] + (7,))
    a0, a1, a2 = drdQ[..., 0], drdQ[..., 1], drdQ[..., 2]
    J[..., 0] = -a1 * qz + a2 * qy
    J[..., 1] = a0 * qz - a2 * qx
    J[..., 2] = -a0 * qy + a1 * qx
    J[..., 3:6] = drdQ
    J[..., 6] = r1 * nQ / (s * Qzs)
    psi, w = robust(np.where(ok, r, 0.0), ap["robust"], ap["robust_scale"])
    Wt = np.where(ok, c2 * w, 0.0).ravel()
    Jv = np.where(ok[..., None], J, 0.0).reshape(-1, 7)
    rv = np.where(ok, r, 0.0).ravel()
    Hm = np.einsum("n,ni,nj->ij", Wt, Jv, Jv)
    g = np.einsum("n,ni,n->i", Wt, Jv, rv)
    cost = float(np.where(ok, c2 * psi, 0.0).sum())
    return Hm, g, cost, int(ok.sum()), rv, Jv, ok


def align_pair_sim3(ap, rho1, rho2, conf2, pose0, s0):
    """Levenberg-Marquardt on (T, s) (sec. III-B, Eq. 12 "optimized using Levenberg-Marquardt"):
    each of ap['gn_steps'] evaluations tries the step solving (H + lambda diag(H)) d = -g at
    the last accepted state; a trial with a lower cost is accepted (lambda / 10), otherwise
    rejected (lambda * 10); lambda starts at 1e-4.  The covariance of (T, log s) is H^-1 at the
    accepted state (7x7).  Returns (pose, s, cov, stats [cost0, cost, count, accepted steps],
    status)."""
    nrm, nvalid = normals(rho1, ap["fx"], ap["fy"], ap["cx"], ap["cy"], ap["normal_disc_rel"])
    pose = np.asarray(pose0, dtype=np.float64).copy()
    s = float(s0)
    Hm, g, cost, cnt = linearize_sim3(ap, rho1, nrm, nvalid, rho2, conf2, pose, s)
    cost0 = cost
    lam = LM_LAMBDA0
    accepted = 0
    status = 0
    for _ in range(ap["gn_steps"]):
        A = Hm + lam * np.diag(np.diag(Hm))
        d = cholesky_solve(A, -g)
        if d is None:
            status = ESINGULAR
            break
        tp = geo.left_update(pose, d[:6])
        ts = s * np.exp(d[6])
        Ht, gt, ct, nt = linearize_sim3(ap, rho1, nrm, nvalid, rho2, conf2, tp, ts)
        if ct < cost:
            pose, s, Hm, g, cost, cnt = tp, ts, Ht, gt, ct, nt
            lam = max(lam / 10.0, LM_LAMBDA_MIN)
            accepted += 1
        else:
            lam = min(lam * 10.0, LM_LAMBDA_MAX)
    cov = np.full((7, 7), np.nan)
    if status == 0:
        cols = [cholesky_solve(Hm, e) for e in np.eye(7)]
        if any(c is None for c in cols):
            status = ESINGULAR
        else:
            cov = np.array(cols).T
    return pose, s, cov, np.array([cost0, cost, cnt, accepted], dtype=np.float64), status


def align_sim3(ap, idepth1, idepth2, conf2, pose_inout, scale_inout):
    """All pairs: updates pose_inout [n][6] and scale_inout [n]; returns cov [n][49],
    stats [n][4], status [n]."""
    n = len(idepth1)
    cov = np.zeros((n, 49))
    stats = np.zeros((n, 4))
    status = np.zeros(n, dtype=np.int32)
    for i in range(n):
        p, s, c, st, code = align_pair_sim3(ap, idepth1[i], idepth2[i], conf2[i], pose_inout[i], scale_inout[i])
        pose_inout[i] = p
        scale_inout[i] = s
        cov[i] = c.ravel()
        stats[i] = st
        status[i] = code
    return cov, stats, status
