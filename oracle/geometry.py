"""Rigid motion, reprojection and flow sampling in FP64 (test infrastructure).

Pose 6-vector (w, t): X_cam = R(w) X_ref + t with R(w) = exp([w]x) (Rodrigues).
The paper leaves the pose convention to the VOLDOR framework (sec. III-A); this
is a reading.  Pose updates are left-multiplicative on SO(3) x R^3:
  (R, t) <- (exp([dw]x) R, exp([dw]x) t + dv).
"""
import numpy as np


def hat(w):
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_so3(w):
    """Rodrigues: R = I + sin(th)/th [w]x + (1 - cos th)/th^2 [w]x^2."""
    w = np.asarray(w, dtype=np.float64)
    th2 = float(w @ w)
    th = np.sqrt(th2)
    K = hat(w)
    if th < 1e-4:
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
    else:
        a = np.sin(th) / th
        b = (1.0 - np.cos(th)) / th2
    return np.eye(3) + a * K + b * (K @ K)


def log_so3(R):
    """Inverse of exp_so3 for rotation angles in [0, pi]."""
    R = np.asarray(R, dtype=np.float64)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])  # 2 sin(th) axis
    s = np.linalg.norm(v)
    c = np.trace(R) - 1.0                                                      # 2 cos(th)
    th = np.arctan2(s, c)
    if c > -1.9:
        if th < 1e-4:
            return v * (0.5 + th * th / 12.0)
        return v * (th / s)
    # near pi: R ~ -I + 2 a a^T (+ small skew part)
    S = 0.5 * (R + R.T)
    B = (S - np.cos(th) * np.eye(3)) / (1.0 - np.cos(th))   # = a a^T
    i = int(np.argmax(np.diag(B)))
    a = B[:, i] / np.sqrt(B[i, i])
    if a @ v < 0:
        a = -a
    return a * th


def pose_rt(p):
    p = np.asarray(p, dtype=np.float64)
    return exp_so3(p[:3]), p[3:6].copy()


def left_update(p, delta):
    """Pose 6-vector after (R, t) <- (exp([dw]x) R, exp([dw]x) t + dv)."""
    R, t = pose_rt(p)
    E = exp_so3(delta[:3])
    R2 = E @ R
    t2 = E @ t + np.asarray(delta[3:6], dtype=np.float64)
    return np.concatenate([log_so3(R2), t2])


def rays(u, v, fx, fy, cx, cy):
    """Normalised rays x~ = K^-1 [u, v, 1] for pixel coordinates (arrays)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    return np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)


def scaled_point(R, t, xt, rho):
    """rho * (R X + t) with X = x~/rho, i.e. R x~ + rho t.  Projection is invariant to
    the scale, so 1/rho never appears (it cancels; sec. III-A Eq. 1 reprojection)."""
    return xt @ R.T + np.asarray(rho, dtype=np.float64)[..., None] * t


def project(Q, fx, fy, cx, cy):
    """Pinhole projection of (scaled) camera points; also returns z > 0."""
    z = Q[..., 2]
    ok = z > 0
    zs = np.where(ok, z, 1.0)
    return fx * Q[..., 0] / zs + cx, fy * Q[..., 1] / zs + cy, ok


def bilinear(field, x, y):
    """Bilinear sample of field [H][W][C] at real coordinates.

    Defined on 0 <= x <= W-1, 0 <= y <= H-1 with integer pixel centres; the right /
    lower tap index is clamped at the far edge (its weight is 0 there).  The sample is
    valid when the point is inside and all four taps are finite.  Returns (value [..., C],
    valid)."""
    H, W = field.shape[:2]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    inside = (x >= 0) & (x <= W - 1) & (y >= 0) & (y <= H - 1)
    xs = np.where(inside, x, 0.0)
    ys = np.where(inside, y, 0.0)
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    ax = (xs - x0)[..., None]
    ay = (ys - y0)[..., None]
    f = field.astype(np.float64)
    a, b, c, d = f[y0, x0], f[y0, x1], f[y1, x0], f[y1, x1]
    val = (1 - ay) * ((1 - ax) * a + ax * b) + ay * ((1 - ax) * c + ax * d)
    fin = (np.isfinite(a) & np.isfinite(b) & np.isfinite(c) & np.isfinite(d)).all(-1)
    return val, inside & fin
