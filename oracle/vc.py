"""Visibility-coverage (VC) scores for VO stride and keyframe selection, FP64 (test
infrastructure).

Sec. III-A "VO Stride and Keyframe Selection" (with its VC equation): for two frames with
known poses, only the first carrying a depth map,
  visibility = share of frame 1's depth pixels whose projection lies inside frame 2's image;
  coverage   = share of frame 2's image area covered by those projections;
  VC         = 2 / (visibility^-1 + coverage^-1), the harmonic mean.
The first frame of a batch whose VC with the batch reference falls below tau_stride becomes
the next batch's reference; the reference becomes a keyframe when its VC with the latest
keyframe falls below tau_keyframe.

Readings (the paper gives no discretisation):
  * a depth pixel is a pixel with finite inverse depth rho > 0 (and, when a confidence map
    is given, confidence >= conf_min);
  * its projection is pi(R x~/rho + t) for the pose (w, t) mapping frame-1 points to frame 2,
    in front of camera 2 (Q_z > 0); it lies inside when its nearest pixel
    (floor(x + 1/2), floor(y + 1/2)) is in [0, W-1] x [0, H-1];
  * frame 2's area is split into cells of c x c pixels (ragged at the far edges); a cell is
    covered when at least one projection's nearest pixel falls in it; coverage is the share
    of covered cells.  Cells larger than one pixel keep coverage from counting the gaps that
    magnification (forward motion) opens between neighbouring projections;
  * VC is 0 when visibility or coverage is 0.
The projection is evaluated in FP64 on both sides of the parity tests, so the inside and
cell decisions agree exactly.
"""
import numpy as np

from . import geometry as geo

N_OUT = 5      # visibility, coverage, VC, visible depth pixels, covered cells


def cells(H, W, c):
    return (H + c - 1) // c, (W + c - 1) // c


def vc_pair(prm, idepth, conf, pose):
    """(visibility, coverage, VC, visible count, covered cells) for one pose."""
    H, W, c = prm["H"], prm["W"], prm["cell"]
    rho = np.asarray(idepth, dtype=np.float64)
    depth = np.isfinite(rho) & (rho > 0)
    if conf is not None:
        depth &= np.asarray(conf, dtype=np.float64) >= prm["conf_min"]
    V, U = np.nonzero(depth)
    n_depth = V.size
    R, t = geo.pose_rt(pose)
    xt = geo.rays(U, V, prm["fx"], prm["fy"], prm["cx"], prm["cy"])
    Q = geo.scaled_point(R, t, xt, rho[V, U])             # rho (R X + t)
    x, y, front = geo.project(Q, prm["fx"], prm["fy"], prm["cx"], prm["cy"])
    xn, yn = np.floor(x + 0.5), np.floor(y + 0.5)
    inside = front & (xn >= 0) & (xn <= W - 1) & (yn >= 0) & (yn <= H - 1)
    n_vis = int(inside.sum())
    hc, wc = cells(H, W, c)
    hit = np.zeros((hc, wc), dtype=bool)
    hit[(yn[inside] // c).astype(np.int64), (xn[inside] // c).astype(np.int64)] = True
    n_cov = int(hit.sum())
    vis = n_vis / n_depth if n_depth else 0.0
    cov = n_cov / (hc * wc)
    vc = 2.0 / (1.0 / vis + 1.0 / cov) if vis > 0 and cov > 0 else 0.0
    return np.array([vis, cov, vc, n_vis, n_cov], dtype=np.float64)


def vc_scores(prm, idepth, conf, poses, tau):
    """Scores of frame 1 against every pose [n][6]; and the index of the first pose whose VC
    is below tau (n when none is): the next batch's reference for tau = tau_stride, or the
    keyframe decision (index 0) for a single pose and tau = tau_keyframe."""
    poses = np.asarray(poses, dtype=np.float64).reshape(-1, 6)
    out = np.stack([vc_pair(prm, idepth, conf, p) for p in poses]) if len(poses) else np.zeros((0, N_OUT))
    below = np.nonzero(out[:, 2] < tau)[0]
    return out, int(below[0]) if below.size else len(poses)
