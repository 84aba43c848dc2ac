"""The input generator's initial-pose recipe (CPU): the street recipe's initial-pose error is
held constant in pixels, so its angular and relative-translation bounds shrink by
f_640 / f above the 640x480 street camera."""
import numpy as np

from paper_2104_06800_amd import synth

F640 = 720.0 * 640 / 1216


def _rot_err_deg(a, b):
    """Per-axis bound check needs R_init R_gt^T; the perturbation is R_init = exp([dw]) R_gt."""
    Ra = synth._rot(a[:3])
    Rb = synth._rot(b[:3])
    dw = synth._rotvec(Ra @ Rb.T)
    return np.degrees(np.abs(dw))


def _bounds(w):
    gt, init = np.asarray(w["pose_gt"]), np.asarray(w["pose_init"])
    rot = max(_rot_err_deg(i, g).max() for i, g in zip(init, gt))
    rel = max(np.linalg.norm(i[3:] - g[3:]) / np.linalg.norm(g[3:]) for i, g in zip(init, gt))
    return rot, rel


def test_street_initial_pose_error_scales_with_focal_length():
    for W, H in ((1216, 352), (640, 480)):
        f = 720.0 * W / 1216
        scale = min(1.0, F640 / f)
        for k in range(3):
            w = synth.make_window(2, k, H=H, W=W, N=3)
            rot, rel = _bounds(w)
            # the bounds hold per axis (exp of a small axis-aligned perturbation composes to
            # within second order of the per-axis draw)
            assert rot <= 0.5 * scale * 1.01 + 1e-9, (W, k, rot)
            assert rel <= 0.05 * scale + 1e-12, (W, k, rel)


def test_small_street_windows_keep_the_base_bounds():
    # at or below 640 px wide the focal length is at most f_640: scale 1
    w = synth.make_window(2, 0, H=48, W=160, N=3)
    assert min(1.0, F640 / (720.0 * 160 / 1216)) == 1.0
    rot, rel = _bounds(w)
    assert rot <= 0.5 * 1.01 and rel <= 0.05
