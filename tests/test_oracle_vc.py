"""Pins of the oracle's visibility-coverage scores (sec. III-A "VO Stride and Keyframe
Selection") on scenes whose answer is fixed by elementary geometry: a fronto-parallel
plane moved sideways by a whole number of pixels, towards and away from the camera, behind
it, with holes and a confidence threshold."""
import numpy as np
import pytest

from oracle import vc


def params(H=24, W=40, cell=4, f=30.0, **kw):
    p = dict(H=H, W=W, fx=f, fy=f, cx=(W - 1) / 2, cy=(H - 1) / 2, cell=cell, conf_min=0.0)
    p.update(kw)
    return p


def harmonic(a, b):
    return 0.0 if a == 0 or b == 0 else 2 * a * b / (a + b)


def plane(p, rho):
    return np.full((p["H"], p["W"]), rho)


def test_identity_pose_sees_and_covers_everything():
    p = params()
    out, first = vc.vc_scores(p, plane(p, 0.3), None, np.zeros((1, 6)), 0.5)
    np.testing.assert_array_equal(out[0], [1.0, 1.0, 1.0, p["H"] * p["W"], 6 * 10])
    assert first == 1


@pytest.mark.parametrize("s,cell", [(1, 4), (7, 4), (13, 1), (16, 8), (39, 2)])
def test_sideways_shift_by_whole_pixels(s, cell):
    """Moving camera 2 so that the plane shifts by s pixels (x2 = x1 + f t_x rho): W - s
    columns stay inside, and frame 2's cell columns from floor(s / c) on are covered."""
    p = params(cell=cell)
    rho = 0.25
    pose = np.array([0, 0, 0, s / (p["fx"] * rho), 0, 0])
    out, _ = vc.vc_scores(p, plane(p, rho), None, pose, 0.0)
    W, H = p["W"], p["H"]
    wc, hc = -(-W // cell), -(-H // cell)
    vis = (W - s) / W
    cov = (wc - s // cell) / wc
    np.testing.assert_allclose(out[0], [vis, cov, harmonic(vis, cov), (W - s) * H, (wc - s // cell) * hc],
                               rtol=1e-15)


def test_forward_motion_magnifies():
    """Camera 2 closer to the plane by dz: projections spread by m = Z / (Z - dz) about the
    principal point; columns with |m (x - cx)| < W/2 stay inside, and with m below the cell
    size every cell of frame 2 is covered."""
    p = params(H=30, W=48, cell=4)
    Z, dz = 4.0, 1.0
    m = Z / (Z - dz)
    out, _ = vc.vc_scores(p, plane(p, 1 / Z), None, np.array([0, 0, 0, 0, 0, -dz]), 0.0)
    cols = sum(1 for x in range(p["W"]) if -0.5 <= p["cx"] + m * (x - p["cx"]) < p["W"] - 0.5)
    rows = sum(1 for y in range(p["H"]) if -0.5 <= p["cy"] + m * (y - p["cy"]) < p["H"] - 0.5)
    vis = cols * rows / (p["W"] * p["H"])
    assert abs(vis - 1 / m ** 2) < 0.05
    np.testing.assert_allclose(out[0][:3], [vis, 1.0, harmonic(vis, 1.0)], rtol=1e-15)


def test_backward_motion_shrinks():
    """Camera 2 farther from the plane: everything stays visible and covers the cells
    between the projections of the image corners."""
    p = params(H=30, W=48, cell=4)
    Z, dz = 4.0, 2.0
    m = Z / (Z + dz)
    out, _ = vc.vc_scores(p, plane(p, 1 / Z), None, np.array([0, 0, 0, 0, 0, dz]), 0.0)
    c = p["cell"]
    xs = [int(np.floor(p["cx"] + m * (x - p["cx"]) + 0.5)) for x in (0, p["W"] - 1)]
    ys = [int(np.floor(p["cy"] + m * (y - p["cy"]) + 0.5)) for y in (0, p["H"] - 1)]
    covered = (xs[1] // c - xs[0] // c + 1) * (ys[1] // c - ys[0] // c + 1)
    cov = covered / (12 * 8)
    np.testing.assert_allclose(out[0], [1.0, cov, harmonic(1.0, cov), p["W"] * p["H"], covered], rtol=1e-15)


def test_points_behind_camera_two_are_not_visible():
    p = params()
    out, first = vc.vc_scores(p, plane(p, 0.5), None, np.array([0, 0, 0, 0, 0, -3.0]), 0.5)
    np.testing.assert_array_equal(out[0], [0.0, 0.0, 0.0, 0.0, 0.0])
    assert first == 0


def test_holes_and_confidence_limit_the_depth_pixels():
    """Holes (NaN, rho <= 0) and pixels under the confidence threshold are not depth
    pixels: visibility counts only the rest, coverage only their cells."""
    p = params(cell=4, conf_min=0.5)
    rho = plane(p, 0.3)
    rho[:, :20] = np.nan              # left half: no depth
    rho[0, 30] = -1.0
    conf = np.ones_like(rho)
    conf[12:, :] = 0.2                # lower half: not confident
    out, _ = vc.vc_scores(p, rho, conf, np.zeros((1, 6)), 0.0)
    n_depth = 12 * 20 - 1
    assert out[0][3] == n_depth and out[0][0] == 1.0
    assert out[0][4] == 3 * 5 and out[0][1] == 15 / 60


def test_first_pose_below_threshold():
    """Growing sideways shifts give falling VC; the first below tau is the next reference."""
    p = params(cell=4)
    rho = 0.25
    shifts = [0, 4, 10, 17, 25, 33]
    poses = np.array([[0, 0, 0, s / (p["fx"] * rho), 0, 0] for s in shifts])
    out, first = vc.vc_scores(p, plane(p, rho), None, poses, 0.6)
    W = p["W"]
    vcs = [harmonic((W - s) / W, (10 - s // 4) / 10) for s in shifts]
    np.testing.assert_allclose(out[:, 2], vcs, rtol=1e-15)
    assert first == next(i for i, v in enumerate(vcs) if v < 0.6)
    assert vc.vc_scores(p, plane(p, rho), None, poses[:2], 0.6)[1] == 2
