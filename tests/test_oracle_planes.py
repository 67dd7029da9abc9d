"""Pins of the oracle's plane-set construction (bounding planes and the
cross-ratio sampling steps, Alg. 2)."""
import numpy as np
import pytest


K = np.array([[800.0, 0, 480], [0, 800.0, 270], [0, 0, 1]])
W, H = 960, 540


def _project_plane(K, R, t, n, delta, u, v):
    """Image in view k of the point where the reference ray through (u, v)
    meets the plane n.X + delta = 0 (independent of the oracle)."""
    r = np.linalg.solve(K, [u, v, 1.0])
    X = -delta / (n @ r) * r
    Y = R @ X + t
    p = K @ Y
    return p[:2] / p[2]


def test_bounding_planes_fronto_equal_depth_range(orc):
    lo, hi = orc.bounding_planes(K, W, H, [0, 0, -1.0], 20.0, 400.0)
    assert (lo, hi) == (20.0, 400.0)


def test_bounding_planes_slanted(orc):
    n = np.array([0.0, -np.sin(0.5), -np.cos(0.5)])
    lo, hi = orc.bounding_planes(K, W, H, n, 20.0, 400.0)
    Ki = np.linalg.inv(K)
    corners = [(0, 0), (W, 0), (0, H), (W, H)]
    a = [abs(n @ (Ki @ [u, v, 1.0])) for u, v in corners]
    assert np.isclose(lo, 20.0 * min(a), rtol=1e-14)
    assert np.isclose(hi, 400.0 * max(a), rtol=1e-14)


@pytest.mark.parametrize("t", [np.array([-3.0, 0.0, 0.0]), np.array([2.0, -1.5, 0.4]),
                               np.array([0.5, 0.2, -1.0])])
def test_cross_ratio_steps_are_one_pixel(orc, t):
    a = 0.03
    R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    n = np.array([0.0, 0.0, -1.0])
    d = orc.cross_ratio_planes(K, W, H, R, t, n, 20.0, 400.0)
    assert d[0] == 400.0 and d[-1] == 20.0
    assert np.all(np.diff(d) < 0)
    # the corner whose images on the bounding planes lie farthest apart
    corners = [(0.5, 0.5), (W - 0.5, 0.5), (0.5, H - 0.5), (W - 0.5, H - 0.5)]
    segs = [np.linalg.norm(_project_plane(K, R, t, n, 20.0, u, v) - _project_plane(K, R, t, n, 400.0, u, v))
            for u, v in corners]
    u, v = corners[int(np.argmax(segs))]
    pts = np.array([_project_plane(K, R, t, n, dd, u, v) for dd in d])
    steps = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    assert np.allclose(steps[:-1], 1.0, atol=1e-6)
    assert 0 < steps[-1] <= 1.0 + 1e-9
    assert len(d) == int(np.floor(max(segs))) + 1 + (1 if np.floor(max(segs)) < max(segs) else 0)


def test_cross_ratio_lateral_translation_is_inverse_uniform(orc):
    """Translation parallel to the image plane and fronto-parallel planes:
    the image motion is f b / delta, so one-pixel steps are uniform in
    inverse distance with step 1 / (f b)."""
    t = np.array([-2.5, 0.0, 0.0])
    d = orc.cross_ratio_planes(K, W, H, np.eye(3), t, [0, 0, -1.0], 20.0, 400.0)
    inv = 1.0 / d[:-1]
    assert np.allclose(np.diff(inv), 1.0 / (800.0 * 2.5), rtol=1e-9, atol=0)


def test_cross_ratio_count_scales_with_baseline(orc):
    n = [0, 0, -1.0]
    c1 = len(orc.cross_ratio_planes(K, W, H, np.eye(3), np.array([-1.0, 0, 0]), n, 20.0, 400.0))
    c2 = len(orc.cross_ratio_planes(K, W, H, np.eye(3), np.array([-2.0, 0, 0]), n, 20.0, 400.0))
    assert abs(c2 - 1 - 2 * (c1 - 1)) <= 2
    with pytest.raises(OverflowError):
        orc.cross_ratio_planes(K, W, H, np.eye(3), np.array([-20.0, 0, 0]), n, 20.0, 400.0, max_planes=256)


def test_cross_ratio_rejects_camera_behind_nearest_plane(orc):
    with pytest.raises(ValueError):
        orc.cross_ratio_planes(K, W, H, np.eye(3), np.array([0, 0, -30.0]), [0, 0, -1.0], 20.0, 400.0)
