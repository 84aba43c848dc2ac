"""Seeded synthetic inputs: scenes, optical-flow windows, depth priors, keyframe pairs.

This module produces *inputs only*.  It ray-casts analytic scenes (infinite
planes, finite quads, spheres) under known rigid camera and object motion,
turns the hits into dense optical flow between successive frames, corrupts the
flow with log-logistic (Fisk) end-point noise and uniform-disc outliers, and
derives noisy depth priors and perturbed initial poses.  It scores, estimates
or aligns nothing, and neither the CPU oracle nor the GPU library import it;
tests and the benchmark hand its arrays to both.

Conventions shared with the consumers (they are properties of the data):
  * world coordinates are the reference camera's (frame 0): x right, y down,
    z forward; pixel (u, v) sits at integer coordinates;
  * a pose 6-vector (w, t) maps reference-camera points to camera f as
    X_f = exp([w]x) X_ref + t;
  * flow[t-1] (t = 1..N) is the displacement from frame t-1 to frame t,
    sampled on frame t-1's pixel grid, (du, dv) interleaved;
  * inverse depth = 1 / z of the reference camera.

Seeds: window k of workload c uses numpy's PCG64 seeded with 1_000_000 * c + k.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

NEAR = 0.05          # metres; hits closer than this are ignored
OUTLIER_RADIUS = 8.0  # px; radius of the uniform disc outlier flows are drawn from


# --------------------------------------------------------------------------- #
# rigid motions (scipy does the exponential / logarithm maps)
# --------------------------------------------------------------------------- #
def _rot(w):
    return Rotation.from_rotvec(np.asarray(w, dtype=np.float64)).as_matrix()


def _rotvec(R):
    return Rotation.from_matrix(R).as_rotvec()


def _compose(A, B):
    """(R, t) of A o B for world->camera transforms."""
    return A[0] @ B[0], A[0] @ B[1] + A[1]


def _as6(T):
    return np.concatenate([_rotvec(T[0]), T[1]])


def _from6(p):
    p = np.asarray(p, dtype=np.float64)
    return _rot(p[:3]), p[3:].copy()


# --------------------------------------------------------------------------- #
# scene description and ray casting
# --------------------------------------------------------------------------- #
@dataclass
class Scene:
    planes_n: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    planes_d: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    quads: list = field(default_factory=list)     # dicts: c, a1, a2, h1, h2, dyn (index or -1)
    spheres_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    spheres_r: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    # per dynamic object: list over frames of (R, t) rest->world
    dyn_motion: list = field(default_factory=list)


def _rays(H, W, fx, fy, cx, cy, T):
    """World-space ray origin and per-pixel directions whose z-parameter is camera depth."""
    R, t = T
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    xc = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], axis=-1)
    d = xc @ R          # R^T x  for row vectors
    o = -R.T @ t
    return o, d


def _raycast(scene: Scene, frame: int, H, W, intr, T):
    """Nearest hit per pixel: camera depth, object id (-1 none, dyn objects >= 1000), world point."""
    fx, fy, cx, cy = intr
    o, d = _rays(H, W, fx, fy, cx, cy, T)
    best = np.full((H, W), np.inf)
    obj = np.full((H, W), -1, dtype=np.int64)
    for i in range(len(scene.planes_d)):
        n = scene.planes_n[i]
        den = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = (scene.planes_d[i] - n @ o) / den
        ok = (lam > NEAR) & (lam < best)
        best = np.where(ok, lam, best)
        obj = np.where(ok, i, obj)
    for qi, q in enumerate(scene.quads):
        c, a1, a2 = q["c"], q["a1"], q["a2"]
        if q["dyn"] >= 0:
            Rm, tm = scene.dyn_motion[q["dyn"]][frame]
            c, a1, a2 = Rm @ c + tm, Rm @ a1, Rm @ a2
        m = np.cross(a1, a2)
        den = d @ m
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = (m @ (c - o)) / den
        X = o + lam[..., None] * d
        rel = X - c
        inside = (np.abs(rel @ a1) <= q["h1"]) & (np.abs(rel @ a2) <= q["h2"])
        ok = inside & (lam > NEAR) & (lam < best)
        best = np.where(ok, lam, best)
        obj = np.where(ok, (1000 + q["dyn"]) if q["dyn"] >= 0 else (100 + qi), obj)
    for si in range(len(scene.spheres_r)):
        c, r = scene.spheres_c[si], scene.spheres_r[si]
        oc = o - c
        a = np.einsum("hwk,hwk->hw", d, d)
        b = 2.0 * (d @ oc)
        cc = oc @ oc - r * r
        disc = b * b - 4 * a * cc
        with np.errstate(invalid="ignore"):
            lam = (-b - np.sqrt(disc)) / (2 * a)
        ok = (disc >= 0) & (lam > NEAR) & (lam < best)
        best = np.where(ok, lam, best)
        obj = np.where(ok, 500 + si, obj)
    X = o + best[..., None] * d
    return best, obj, X


def _advect(scene: Scene, obj, X, f0, f1):
    """World position at frame f1 of surface points seen at frame f0."""
    Y = X.copy()
    for k in range(len(scene.dyn_motion)):
        m = obj == 1000 + k
        if not m.any():
            continue
        R0, t0 = scene.dyn_motion[k][f0]
        R1, t1 = scene.dyn_motion[k][f1]
        rest = (X[m] - t0) @ R0           # R0^T (X - t0)
        Y[m] = rest @ R1.T + t1
    return Y


def _project(X, T, intr):
    fx, fy, cx, cy = intr
    R, t = T
    Xc = X @ R.T + t
    z = Xc[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * Xc[..., 0] / z + cx
        v = fy * Xc[..., 1] / z + cy
    return u, v, z


# --------------------------------------------------------------------------- #
# noise
# --------------------------------------------------------------------------- #
def fisk_noise(rng, shape, alpha, beta):
    """2-vectors whose length is log-logistic(alpha, beta) by inverse CDF and whose angle is uniform."""
    u = rng.uniform(1e-12, 1 - 1e-12, size=shape)
    r = alpha * (u / (1.0 - u)) ** (1.0 / beta)
    phi = rng.uniform(0, 2 * np.pi, size=shape)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=-1)


def disc_outliers(rng, shape, radius=OUTLIER_RADIUS):
    """2-vectors uniform in a disc."""
    r = radius * np.sqrt(rng.uniform(0, 1, size=shape))
    phi = rng.uniform(0, 2 * np.pi, size=shape)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=-1)


def stereo_prior(rng, rho_gt, fb, alpha_px=0.6, beta=1.0, outlier_frac=0.08, hole_frac=0.05):
    """An external stereo depth prior of a window's reference frame: disparity fb * rho_gt plus a
    signed log-logistic(alpha_px, beta) error (inverse CDF, random sign), a fraction replaced by
    disparities uniform over [0, fb * max(rho_gt)] (matching failures), a fraction of holes (NaN);
    returned as inverse depth [1][H][W] with the window fields of the empirical disparity model."""
    shape = rho_gt.shape
    u = rng.uniform(1e-12, 1 - 1e-12, size=shape)
    mag = alpha_px * (u / (1.0 - u)) ** (1.0 / beta)
    d = fb * rho_gt + np.where(rng.uniform(size=shape) < 0.5, -mag, mag)
    D = float(fb * np.nanmax(rho_gt))
    out = rng.uniform(size=shape) < outlier_frac
    d = np.where(out, rng.uniform(0.0, D, size=shape), d)
    pr = np.maximum(d, 1e-3) / fb
    pr[rng.uniform(size=shape) < hole_frac] = np.nan
    fields = dict(prior_model=1, prior_disp_scale=float(fb), prior_sigma_rel=float(alpha_px),
                  prior_fisk_beta=float(beta), prior_uniform_rel=D)
    return pr[None].astype(np.float32), fields


# --------------------------------------------------------------------------- #
# scene recipes
# --------------------------------------------------------------------------- #
def _random_dir_near_axis(rng, max_deg):
    th = np.deg2rad(max_deg) * np.sqrt(rng.uniform(0, 1))
    ph = rng.uniform(0, 2 * np.pi)
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)])


def scene_planes(rng, n_planes, H, W, intr, rho_lo, rho_hi, max_tilt_deg=30.0):
    """Infinite planes, normals within max_tilt of the optical axis, each through an anchor
    pixel at inverse depth U[rho_lo, rho_hi]; plus a fronto-parallel backstop far away."""
    fx, fy, cx, cy = intr
    ns, ds = [], []
    for _ in range(n_planes):
        n = _random_dir_near_axis(rng, max_tilt_deg)
        ua, va = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        rho = rng.uniform(rho_lo, rho_hi)
        A = np.array([(ua - cx) / fx, (va - cy) / fy, 1.0]) / rho
        ns.append(n)
        ds.append(n @ A)
    ns.append(np.array([0.0, 0.0, -1.0]))
    ds.append(-1.0 / (0.8 * rho_lo))
    return Scene(planes_n=np.array(ns), planes_d=np.array(ds))


def _quad(c, yaw_deg, pitch_deg, h1, h2, dyn=-1):
    R = _rot([np.deg2rad(pitch_deg), np.deg2rad(yaw_deg), 0.0])
    return {"c": np.asarray(c, float), "a1": R @ np.array([1.0, 0, 0]),
            "a2": R @ np.array([0, 1.0, 0]), "h1": float(h1), "h2": float(h2), "dyn": dyn}


def scene_street(rng, n_frames, n_quads=27, n_bumps=10, n_dyn=5, dyn_frac=0.15, intr=None, HW=None):
    """Forward-driving street: ground, two walls, a far backdrop (30 planar surfaces with
    the quads), spherical bumps, and n_dyn moving fronto-parallel boxes covering about
    dyn_frac of the reference image."""
    H, W = HW
    fx, fy, cx, cy = intr
    wl, wr = rng.uniform(5, 9), rng.uniform(5, 9)
    ns = [np.array([0.0, -1.0, 0.0]), np.array([1.0, 0, 0]), np.array([-1.0, 0, 0]),
          np.array([0.0, 0, -1.0])]
    ds = [-1.6, -wl, -wr, -150.0]
    quads = []
    for _ in range(n_quads):
        side = rng.choice([-1, 1])
        x = side * rng.uniform(2.5, 0.9 * (wl if side < 0 else wr))
        quads.append(_quad([x, rng.uniform(-1.5, 1.0), rng.uniform(14, 90)],
                           rng.uniform(-40, 40), rng.uniform(-10, 10),
                           rng.uniform(0.5, 3.0), rng.uniform(0.4, 2.0)))
    sc = []
    sr = []
    for _ in range(n_bumps):
        r = rng.uniform(0.4, 1.8)
        side = rng.choice([-1, 1])
        sc.append([side * rng.uniform(2.0, 5.0), 1.6 - 0.4 * r, rng.uniform(16, 80)])
        sr.append(r)
    # moving boxes: pixel area per box ~ dyn_frac/n_dyn of the image
    motion = []
    area = 1.8 * dyn_frac * H * W / n_dyn   # about 45% of it ends up occluded
    for k in range(n_dyn):
        z = rng.uniform(12, 30)
        aspect = rng.uniform(0.8, 1.6)
        wpx = np.sqrt(area * aspect)
        hpx = area / wpx
        hw, hh = 0.5 * wpx * z / fx, 0.5 * hpx * z / fy
        x = rng.uniform(-wl + hw + 0.5, wr - hw - 0.5) if wl + wr > 2 * hw + 1 else 0.0
        c = np.array([x, 1.6 - hh, z])
        quads.append(_quad(c, 0.0, 0.0, hw, hh, dyn=k))
        v = np.array([rng.uniform(-0.6, 0.6), 0.0, rng.uniform(-1.5, 1.5)])
        wv = np.array([0.0, np.deg2rad(rng.uniform(-2, 2)), 0.0])
        frames = []
        for f in range(n_frames + 1):
            Rm = _rot(wv * f)
            frames.append((Rm, c + f * v - Rm @ c))
        motion.append(frames)
    return Scene(planes_n=np.array(ns), planes_d=np.array(ds), quads=quads,
                 spheres_c=np.array(sc, float).reshape(-1, 3), spheres_r=np.array(sr, float),
                 dyn_motion=motion)


def scene_room(rng, intr=None, HW=None, n_quads=8, n_spheres=4):
    """Indoor room: floor, ceiling, three walls, boxes and spheres, depths ~1.5-7 m."""
    ns = [np.array([0.0, -1.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([1.0, 0, 0]),
          np.array([-1.0, 0, 0]), np.array([0.0, 0, -1.0])]
    ds = [-rng.uniform(1.2, 1.6), -rng.uniform(1.2, 1.8), -rng.uniform(2.5, 4.0),
          -rng.uniform(2.5, 4.0), -rng.uniform(5.5, 7.0)]
    quads = [_quad([rng.uniform(-1.8, 1.8), rng.uniform(-0.8, 0.9), rng.uniform(2.5, 5.0)],
                   rng.uniform(-35, 35), rng.uniform(-15, 15),
                   rng.uniform(0.2, 0.7), rng.uniform(0.2, 0.6)) for _ in range(n_quads)]
    sc = [[rng.uniform(-1.5, 1.5), rng.uniform(-0.6, 0.8), rng.uniform(2.5, 5.0)] for _ in range(n_spheres)]
    sr = [rng.uniform(0.2, 0.5) for _ in range(n_spheres)]
    return Scene(planes_n=np.array(ns), planes_d=np.array(ds), quads=quads,
                 spheres_c=np.array(sc, float).reshape(-1, 3), spheres_r=np.array(sr, float))


# --------------------------------------------------------------------------- #
# trajectories
# --------------------------------------------------------------------------- #
def traj_small(rng, N, rot_deg=2.0, trans=0.1):
    """Per-frame increments: rotation U[-rot_deg, rot_deg] per axis, translation of
    random direction and length U[trans/2, trans]."""
    Ts = [(np.eye(3), np.zeros(3))]
    for _ in range(N):
        w = np.deg2rad(rng.uniform(-rot_deg, rot_deg, size=3))
        d = rng.normal(size=3)
        d *= rng.uniform(0.5 * trans, trans) / np.linalg.norm(d)
        Ts.append(_compose((_rot(w), d), Ts[-1]))
    return Ts


def traj_drive(rng, N, tz=(0.5, 1.5), yaw_deg=3.0):
    """Forward driving: the camera advances U[tz] metres along its optical axis per frame
    and yaws by at most yaw_deg."""
    Ts = [(np.eye(3), np.zeros(3))]
    for _ in range(N):
        step = (_rot([0.0, np.deg2rad(rng.uniform(-yaw_deg, yaw_deg)), 0.0]),
                np.array([0.0, 0.0, -rng.uniform(*tz)]))
        Ts.append(_compose(step, Ts[-1]))
    return Ts


def traj_6dof(rng, N, max_deg=5.0, max_t=0.3):
    """Frames spread along a random 6-DoF motion of at most max_deg and max_t metres,
    with small per-frame jitter."""
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    w_end = ax * np.deg2rad(rng.uniform(0.5, 1.0) * max_deg)
    d = rng.normal(size=3)
    t_end = d / np.linalg.norm(d) * rng.uniform(0.5, 1.0) * max_t
    Ts = [(np.eye(3), np.zeros(3))]
    for f in range(1, N + 1):
        a = f / N
        w = a * w_end + np.deg2rad(0.05) * rng.normal(size=3)
        t = a * t_end + 0.005 * rng.normal(size=3)
        Ts.append((_rot(w), t))
    return Ts


def perturb(rng, T, max_deg=0.5, rel_t=0.05):
    """Initial-pose recipe: rotation error U[-max_deg, max_deg] per axis and a translation
    error of length U[0, rel_t] * |t| in a random direction."""
    R, t = T
    dw = np.deg2rad(rng.uniform(-max_deg, max_deg, size=3))
    d = rng.normal(size=3)
    d *= rng.uniform(0, rel_t) * np.linalg.norm(t) / np.linalg.norm(d)
    return _rot(dw) @ R, t + d


# --------------------------------------------------------------------------- #
# window assembly
# --------------------------------------------------------------------------- #
def render_window(scene, Ts, H, W, intr, rng, alpha, beta, noise=True, block_frac=0.0):
    """Flows between successive frames (on frame t-1's grid), reference inverse depth
    and the reference pixels that see moving content."""
    N = len(Ts) - 1
    flow = np.zeros((N, H, W, 2), dtype=np.float64)
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    dyn0 = None
    z0 = None
    bw = bh = 0
    if block_frac > 0:
        bw = int(round(np.sqrt(block_frac * H * W * W / H)))
        bh = int(round(block_frac * H * W / bw))
        bx, by = rng.integers(0, W - bw), rng.integers(0, H - bh)
    for t in range(1, N + 1):
        z, obj, X = _raycast(scene, t - 1, H, W, intr, Ts[t - 1])
        if t == 1:
            z0 = z
            dyn0 = obj >= 1000
        Y = _advect(scene, obj, X, t - 1, t)
        pu, pv, zt = _project(Y, Ts[t], intr)
        f = np.stack([pu - u, pv - v], axis=-1)
        bad = ~np.isfinite(z) | (zt <= NEAR) | ~np.isfinite(f).all(-1)
        if noise:
            f = f + fisk_noise(rng, (H, W), alpha, beta)
        nb = int(bad.sum())
        if nb:
            f[bad] = disc_outliers(rng, (nb,))
        if block_frac > 0:
            if t == 1:
                dyn0 = dyn0.copy()
                dyn0[by:by + bh, bx:bx + bw] = True
            f[by:by + bh, bx:bx + bw] = disc_outliers(rng, (bh, bw))
            bx = int(np.clip(bx + rng.integers(-2, 3), 0, W - bw))
            by = int(np.clip(by + rng.integers(-2, 3), 0, H - bh))
        flow[t - 1] = f
    return flow, 1.0 / z0, dyn0


def default_params(H, W, N, intr, **kw):
    """Window parameters (mirrors the library's window struct)."""
    p = dict(H=H, W=W, N=N, P=0, fx=intr[0], fy=intr[1], cx=intr[2], cy=intr[3],
             fisk_alpha=0.5, fisk_beta=2.0, outlier_density=1.0 / (np.pi * OUTLIER_RADIUS ** 2),
             hmm_gamma=0.9, idepth_min=0.025, idepth_max=1.0, perturb_sigma0=0.3,
             prior_sigma_rel=0.05, prior_uniform_rel=2.0, prior_inlier_default=0.5,
             n_candidates=16, coarse_stride=4, tile=32, pose_gn_steps=2, chain_axis=0,
             seed=0, window_id=0, iters=5)
    p.update(kw)
    return p


def make_window(cfg: int, k: int = 0, noise: bool = True, H=None, W=None, N=None, **kw):
    """One synthetic window of the named workload.

    cfg 1: 64x48, f=50, N=3, 4 random planes, small motion, Fisk(0.5, 2), a 10% outlier
           block, K=16, 5 iterations.
    cfg 2: 1216x352, f=720, N=6, street scene with 15% moving boxes, forward driving,
           Fisk(0.8, 2), K=32, 10 iterations.
    cfg 3: 640x480, f=500, N=8, indoor room, 6-DoF motion <= 5 deg / 0.3 m, Fisk(0.5, 2),
           one depth prior (5% multiplicative noise on depth, 10% holes), K=32, 10 iterations.
    cfg 4: the cfg-2 street recipe at 640x480 (intrinsics scaled), N=6.
    H, W, N override the size (cfg 2/3 recipes scale the intrinsics).
    Initial poses: the true ones with a rotation error of up to 0.5 deg per axis and a
    translation error of up to 5% (perturb); the street recipe shrinks both by
    f_640 / f for focal lengths above f_640 = 720 * 640 / 1216 px, so the initial error
    is the same in pixels as at 640x480.
    """
    rng = np.random.default_rng(1_000_000 * cfg + k)
    pose_scale = 1.0
    if cfg == 1:
        H, W, N = H or 48, W or 64, N or 3
        intr = (50.0 * W / 64, 50.0 * W / 64, W / 2, H / 2)
        scene = scene_planes(rng, 4, H, W, intr, 0.05, 0.5)
        Ts = traj_small(rng, N)
        alpha, beta = 0.5, 2.0
        flow, rho_gt, dyn = render_window(scene, Ts, H, W, intr, rng, alpha, beta, noise,
                                          block_frac=0.10 if noise else 0.0)
        params = default_params(H, W, N, intr, fisk_alpha=alpha, fisk_beta=beta,
                                idepth_min=0.02, idepth_max=1.25, n_candidates=16, iters=5)
    elif cfg in (2, 4):
        if cfg == 2:
            H, W, N = H or 352, W or 1216, N or 6
            f0 = 720.0 * W / 1216
        else:
            H, W, N = H or 480, W or 640, N or 6
            f0 = 720.0 * W / 1216
        intr = (f0, f0, W / 2, H / 2)
        scene = scene_street(rng, N, intr=intr, HW=(H, W))
        pose_scale = min(1.0, (720.0 * 640 / 1216) / f0)
        Ts = traj_drive(rng, N)
        alpha, beta = 0.8, 2.0
        flow, rho_gt, dyn = render_window(scene, Ts, H, W, intr, rng, alpha, beta, noise)
        params = default_params(H, W, N, intr, fisk_alpha=alpha, fisk_beta=beta,
                                idepth_min=0.005, idepth_max=0.5, n_candidates=32, iters=10)
    elif cfg == 3:
        H, W, N = H or 480, W or 640, N or 8
        f0 = 500.0 * W / 640
        intr = (f0, f0, W / 2, H / 2)
        scene = scene_room(rng, intr=intr, HW=(H, W))
        Ts = traj_6dof(rng, N)
        alpha, beta = 0.5, 2.0
        flow, rho_gt, dyn = render_window(scene, Ts, H, W, intr, rng, alpha, beta, noise)
        params = default_params(H, W, N, intr, fisk_alpha=alpha, fisk_beta=beta,
                                idepth_min=0.1, idepth_max=1.0, n_candidates=32, iters=10)
    else:
        raise ValueError(f"unknown workload {cfg}")
    pose_gt = np.stack([_as6(T) for T in Ts[1:]])
    pose_init = np.stack([_as6(perturb(rng, T, max_deg=0.5 * pose_scale, rel_t=0.05 * pose_scale)) for T in Ts[1:]])
    params["seed"] = int(rng.integers(0, 2 ** 63))
    params.update(kw)
    out = dict(params=params, flow=flow.astype(np.float32), pose_gt=pose_gt,
               pose_init=pose_init, idepth_gt=rho_gt, dynamic=dyn, intr=intr)
    if cfg == 3:
        depth = 1.0 / rho_gt
        noisy = depth * (1.0 + 0.05 * rng.normal(size=depth.shape))
        pr = 1.0 / np.maximum(noisy, 1e-3)
        pr[rng.uniform(size=pr.shape) < 0.10] = np.nan
        out["prior_idepth"] = pr[None].astype(np.float32)
        out["prior_pose"] = np.zeros((1, 6))
        params["P"] = 1
    return out


BATCH_SEED = 5_000_000


def batch_shapes(n=64, seed=BATCH_SEED):
    """Shapes of the uneven-window batch: width U{320..1216} and height U{240..352} in steps
    of 16, N U{3..8}; odd windows carry a depth prior (indoor recipe), even ones are street
    windows."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W = int(rng.integers(20, 77)) * 16
        H = int(rng.integers(15, 23)) * 16
        N = int(rng.integers(3, 9))
        out.append((i, H, W, N, bool(i % 2)))
    return out


def batch_window(spec, seed=BATCH_SEED):
    """One window of the uneven batch from its (index, H, W, N, prior) spec."""
    i, H, W, N, prior = spec
    return make_window(3 if prior else 2, seed + i, H=H, W=W, N=N)


def make_pairs(n_pairs: int, H=480, W=640, seed=3_000_000, max_deg=2.0, max_t=0.1,
               noise_rel=0.0, conf="ones", planar=False):
    """Keyframe pairs for point-to-plane alignment: two inverse-depth maps of one room
    scene from cameras related by a random motion (<= max_deg, <= max_t), the confidence
    of map 2 and the true pose of camera 2 relative to camera 1 (maps cam-2 points to
    cam-1 points).  planar=True leaves out the spheres (piecewise-planar scene)."""
    rng = np.random.default_rng(seed)
    f0 = 500.0 * W / 640
    intr = (f0, f0, W / 2, H / 2)
    rho1 = np.zeros((n_pairs, H, W), np.float32)
    rho2 = np.zeros((n_pairs, H, W), np.float32)
    c2 = np.ones((n_pairs, H, W), np.float32)
    obj1 = np.zeros((n_pairs, H, W), np.int64)
    obj2 = np.zeros((n_pairs, H, W), np.int64)
    pose = np.zeros((n_pairs, 6))
    for i in range(n_pairs):
        scene = scene_room(rng, intr=intr, HW=(H, W), n_spheres=0 if planar else 4)
        T1 = (_rot(np.deg2rad(rng.uniform(-3, 3, 3))), rng.uniform(-0.2, 0.2, 3))
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        dT = (_rot(ax * np.deg2rad(rng.uniform(0.3, 1.0) * max_deg)),
              rng.normal(size=3))
        dT = (dT[0], dT[1] / np.linalg.norm(dT[1]) * rng.uniform(0.3, 1.0) * max_t)
        T2 = _compose(dT, T1)
        z1, obj1[i], _ = _raycast(scene, 0, H, W, intr, T1)
        z2, obj2[i], _ = _raycast(scene, 0, H, W, intr, T2)
        r1, r2 = 1.0 / z1, 1.0 / z2
        if noise_rel > 0:
            r2 = r2 * (1.0 + noise_rel * rng.normal(size=r2.shape))
        rho1[i], rho2[i] = r1, r2
        if conf == "random":
            c2[i] = rng.uniform(0.3, 1.0, size=(H, W))
        # cam2 -> cam1:  X1 = R1 R2^T (X2 - t2) + t1
        R21 = T1[0] @ T2[0].T
        pose[i] = _as6((R21, T1[1] - R21 @ T2[1]))
    params = dict(H=H, W=W, fx=intr[0], fy=intr[1], cx=intr[2], cy=intr[3], robust=0,
                  robust_scale=0.02, gn_steps=10, normal_disc_rel=0.05, scale_s=1.0)
    return dict(params=params, idepth1=rho1, idepth2=rho2, conf2=c2, pose_gt=pose, object1=obj1,
                object2=obj2)


def _rel(Ts):
    """Poses of frames 1.. relative to frame 0 (world -> camera each)."""
    R0, t0 = Ts[0]
    inv0 = (R0.T, -R0.T @ t0)
    return [_compose(T, inv0) for T in Ts]


def vo_start(rng, pose6, max_deg=1.0, max_t=0.03):
    """A chained visual-odometry estimate of a relative pose: the 6-vector moved by a random
    left motion of up to max_deg per rotation axis and max_t per translation axis."""
    dT = (_rot(np.deg2rad(rng.uniform(-max_deg, max_deg, 3))), rng.uniform(-max_t, max_t, 3))
    return _as6(_compose(dT, _from6(pose6)))


def keyframe_pair(k, H=480, W=640, N=8, seed=3_500_000):
    """Two indoor windows of one room whose reference cameras are related by a random motion
    (<= 5 deg, <= 0.3 m), each with its flows, depth prior (as workload 3) and perturbed
    initial poses, for keyframe alignment of GEM outputs.  Returns (window a, window b, pose
    of camera b relative to camera a as a 6-vector mapping camera-b points to camera a)."""
    rng = np.random.default_rng(seed + k)
    f0 = 500.0 * W / 640
    intr = (f0, f0, W / 2, H / 2)
    scene = scene_room(rng, intr=intr, HW=(H, W))
    alpha, beta = 0.5, 2.0
    TA = traj_6dof(rng, N)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    d = rng.normal(size=3)
    dT = (_rot(ax * np.deg2rad(rng.uniform(0.5, 1.0) * 5.0)), d / np.linalg.norm(d) * rng.uniform(0.5, 1.0) * 0.3)
    TB = [_compose(T, dT) for T in traj_6dof(rng, N)]
    out = []
    for Ts in (TA, TB):
        flow, rho_gt, dyn = render_window(scene, Ts, H, W, intr, rng, alpha, beta, True)
        rel = _rel(Ts)
        params = default_params(H, W, N, intr, fisk_alpha=alpha, fisk_beta=beta, idepth_min=0.1, idepth_max=1.0,
                                n_candidates=32, iters=10, P=1)
        params["seed"] = int(rng.integers(0, 2 ** 63))
        depth = 1.0 / rho_gt
        pr = 1.0 / np.maximum(depth * (1.0 + 0.05 * rng.normal(size=depth.shape)), 1e-3)
        pr[rng.uniform(size=pr.shape) < 0.10] = np.nan
        out.append(dict(params=params, flow=flow.astype(np.float32),
                        pose_gt=np.stack([_as6(T) for T in rel[1:]]),
                        pose_init=np.stack([_as6(perturb(rng, T)) for T in rel[1:]]),
                        idepth_gt=rho_gt, dynamic=dyn, intr=intr, prior_idepth=pr[None].astype(np.float32),
                        prior_pose=np.zeros((1, 6))))
    # camera b -> camera a:  X_a = R_a0 R_b0^T (X_b - t_b0) + t_a0, with camera a = world
    Rb, tb = TB[0]
    return out[0], out[1], _as6((Rb.T, -Rb.T @ tb))
