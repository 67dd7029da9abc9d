"""Oracle pins: median, normals, normal smoothing, confidence and the
coarse-to-fine seeds (upsampling, sampling windows, surface-normal offsets)."""
import math

import numpy as np
import pytest


def test_median5_matches_library_median(orc):
    rng = np.random.default_rng(0)
    d = rng.random((13, 17)).astype(np.float32)
    d[rng.random(d.shape) < 0.2] = 0.0
    out = orc.median5(d)
    pad = np.pad(d, 2, mode="edge")
    win = np.lib.stride_tricks.sliding_window_view(pad, (5, 5))
    assert np.array_equal(out, np.median(win.reshape(13, 17, 25), axis=-1).astype(np.float32))
    assert np.all(orc.median5(np.full((5, 6), 2.5, np.float32)) == 2.5)


def _plane_depth(Ki, n, c, w, h):
    """Depth map of the plane n^T X + c = 0 (closed form d = -c / n^T K^-1 p)."""
    uu, vv = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    rays = np.stack([uu, vv, np.ones_like(uu)], -1) @ Ki.T
    return (-c / (rays @ n)), rays


def test_normals_of_a_plane(orc):
    K = np.array([[300.0, 0, 40], [0, 300.0, 30], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    rng = np.random.default_rng(1)
    for _ in range(10):
        n = rng.normal(size=3)
        n[2] = -abs(n[2]) - 1.0
        n /= np.linalg.norm(n)
        d, _ = _plane_depth(Ki, n, 50.0, 80, 60)
        assert np.all(d > 0)
        out = orc.normals(d.astype(np.float32), Ki)
        # normal of the plane, facing the camera, at every pixel (float depth)
        assert np.max(np.abs(out.reshape(-1, 3) - n)) < 2e-3
        assert np.allclose(np.linalg.norm(out, axis=-1), 1.0, atol=1e-6)
    # fronto-parallel plane -> (0, 0, -1)
    out = orc.normals(np.full((6, 7), 10.0, np.float32), Ki)
    assert np.allclose(out, [0, 0, -1.0], atol=1e-7)
    # a missing neighbour invalidates the normal
    d = np.full((6, 7), 10.0, np.float32)
    d[3, 3] = 0
    out = orc.normals(d, Ki)
    for (y, x) in ((3, 3), (2, 3), (4, 3), (3, 2), (3, 4)):
        assert np.all(out[y, x] == 0)
    assert np.allclose(out[0, 0], [0, 0, -1.0], atol=1e-7)


def test_normal_smoothing_fixed_points(orc):
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, (12, 14)).astype(np.uint8)
    n = np.array([0.3, -0.2, -0.9])
    n /= np.linalg.norm(n)
    field = np.broadcast_to(n, (12, 14, 3)).astype(np.float32).copy()
    out = orc.normal_smooth(field, img, 2, 10.0)
    assert np.max(np.abs(out - field)) < 1e-6
    # an isolated normal among invalid pixels only keeps itself
    f2 = np.zeros((12, 14, 3), np.float32)
    f2[5, 5] = n
    out = orc.normal_smooth(f2, img, 2, 10.0)
    assert np.allclose(out[5, 5], n, atol=1e-6) and np.count_nonzero(out.any(-1)) == 1


def test_normal_smoothing_weights(orc):
    """Two neighbours: the result is the normalised n_p + w_q n_q with the
    Gaussian-appearance weight of Eq. normal-smooth; check via the angle,
    which depends only on the weight ratio."""
    img = np.zeros((5, 5), np.uint8)
    img[2, 3] = 20                             # intensity step of 20 at q
    f = np.zeros((5, 5, 3), np.float32)
    a = np.array([0.0, 0.0, -1.0])
    b = np.array([1.0, 0.0, 0.0])
    f[2, 2] = a
    f[2, 3] = b
    out = orc.normal_smooth(f, img, 2, 10.0)
    ratio = out[2, 2, 0] / -out[2, 2, 2]       # = w_q / 1
    # sigma = radius = 2, distance 1, dI = 20, beta = 10
    w_q = math.exp(-1 / 8.0 - 2.0) / math.sqrt(2 * math.pi * 4.0)
    assert ratio == pytest.approx(w_q, rel=1e-5)


@pytest.mark.parametrize("radius", [1, 2, 3])
def test_normal_smoothing_on_flat_intensity_is_a_gaussian_correlation(orc, radius):
    """With one intensity everywhere the appearance term is 1 and Eq.
    normal-smooth becomes a correlation of the normal field with the
    Gaussian of sigma = radius over the (2r+1)^2 window, the pixel itself
    taken with weight 1 and neighbours outside the image left out: checked
    against scipy's correlate, then normalised."""
    from scipy import ndimage
    rng = np.random.default_rng(radius)
    h, w = 17, 23
    f = rng.normal(0, 1, (h, w, 3)).astype(np.float32)
    f[..., 2] = -np.abs(f[..., 2]) - 0.5
    f /= np.linalg.norm(f, axis=-1, keepdims=True)
    f[rng.random((h, w)) < 0.1] = 0.0          # invalid normals take no part
    img = np.full((h, w), 77, np.uint8)
    sig = float(radius)
    yy, xx = np.mgrid[-radius:radius + 1, -radius:radius + 1]
    ker = np.exp(-(xx ** 2 + yy ** 2) / (2 * sig * sig)) / math.sqrt(2 * math.pi * sig * sig)
    ker[radius, radius] = 1.0
    acc = np.stack([ndimage.correlate(f[..., c].astype(np.float64), ker, mode="constant", cval=0.0)
                    for c in range(3)], axis=-1)
    valid = np.any(f != 0, axis=-1)
    exp = np.where(valid[..., None], acc / np.linalg.norm(acc, axis=-1, keepdims=True), 0.0)
    got = orc.normal_smooth(f, img, radius, 10.0)
    assert np.max(np.abs(got - exp)) < 2e-6


def test_confidence_closed_forms(orc):
    fam_n = np.array([[0, 0, -1.0]])
    lab = np.zeros((1, 4), np.int32)
    fam = np.zeros((1, 4), np.int32)
    nr = np.zeros((1, 4, 3), np.float32)
    nr[0, 0] = [0, 0, -1]                                           # all aligned -> 1
    t = math.radians(40)
    nr[0, 1] = [math.sin(t), 0, -math.cos(t)]                        # 40 deg -> (cos40-.5)/.5
    t = math.radians(61)
    nr[0, 2] = [math.sin(t), 0, -math.cos(t)]                        # beyond rho -> 0
    c = orc.confidence(nr, lab, fam, fam_n, 60.0)
    assert c[0, 0] == pytest.approx(1.0)
    assert c[0, 1] == pytest.approx((math.cos(math.radians(40)) - 0.5) / 0.5, rel=1e-6)
    assert c[0, 2] == 0 and c[0, 3] == 0
    # slanted sampling plane at 30 deg to the viewing direction, normal equal to it
    s = math.radians(30)
    fam_n2 = np.array([[0, math.sin(s), -math.cos(s)]])
    nr2 = np.zeros((1, 1, 3), np.float32)
    nr2[0, 0] = fam_n2[0]
    c = orc.confidence(nr2, lab[:, :1], fam[:, :1], fam_n2, 60.0)
    assert c[0, 0] == pytest.approx((math.cos(s) - 0.5) / 0.5, rel=1e-6)
    # invalid depth label -> 0
    c = orc.confidence(nr[:, :1], -np.ones((1, 1), np.int32), fam[:, :1], fam_n, 60.0)
    assert c[0, 0] == 0


def test_upsample_nn(orc):
    src = np.arange(12, dtype=np.float32).reshape(3, 4)
    out = orc.upsample_nn(src, 9, 7)
    yy, xx = np.mgrid[0:7, 0:9]
    assert np.array_equal(out, src[np.minimum(yy // 2, 2), np.minimum(xx // 2, 3)])
    src3 = np.random.default_rng(3).random((3, 4, 3)).astype(np.float32)
    out3 = orc.upsample_nn(src3, 8, 6)
    assert np.array_equal(out3, np.repeat(np.repeat(src3, 2, 0), 2, 1))


def test_window_offsets_centre_on_seed(orc):
    K = np.array([[200.0, 0, 20], [0, 200.0, 15], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    G, W = 64, 16
    deltas = orc.plane_list(20.0, 400.0, G)
    rng = np.random.default_rng(4)
    j = rng.integers(0, G, (30, 40))
    dbar = deltas[j].astype(np.float32)
    offs = orc.window_offsets(dbar, Ki, np.array([[0, 0, -1.0]]), [deltas], [W])
    exp = np.clip(j - W // 2, 0, G - W)
    assert np.array_equal(offs[0], exp)
    dbar[0, 0] = 0
    offs = orc.window_offsets(dbar, Ki, np.array([[0, 0, -1.0]]), [deltas], [W])
    assert offs[0, 0, 0] == (G - W) // 2
    # a window covering the whole list starts at 0
    offs = orc.window_offsets(dbar, Ki, np.array([[0, 0, -1.0]]), [deltas], [G])
    assert offs.max() == 0
    # a list of varying spacing (geometric distances): the window of a seed on
    # plane j still starts at j - W/2
    geo = 20.0 * 1.05 ** np.arange(G)
    dbar = geo[j].astype(np.float32)
    offs = orc.window_offsets(dbar, Ki, np.array([[0, 0, -1.0]]), [geo], [W])
    j32 = np.array([np.abs(geo - v).argmin() for v in dbar.astype(np.float64).ravel()]).reshape(j.shape)
    assert np.array_equal(j32, j)
    assert np.array_equal(offs[0], np.clip(j - W // 2, 0, G - W))


def test_delta_i_on_an_analytic_plane(orc):
    """For a seed lying on a plane n^T X + c = 0 with its true normal, 1/depth
    is affine in the pixel, so the fronto-parallel index jump toward q = p - r
    is the constant (n^T K^-1 r) / (c * step); opposite paths get opposite
    jumps (cf. the same magnitude for opposite paths noted by the paper)."""
    K = np.array([[300.0, 0, 40], [0, 300.0, 30], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    n = np.array([0.0, 0.6, -0.8])
    c = 40.0
    d, _ = _plane_depth(Ki, n, c, 80, 60)
    step = (1 / 20 - 1 / 400) / 511
    deltas = orc.plane_list(20.0, 400.0, 512)
    nb = np.broadcast_to(n, (60, 80, 3)).astype(np.float32).copy()
    dI = orc.delta_i(d.astype(np.float32), nb, Ki, np.array([[0, 0, -1.0]]), [deltas])
    DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]
    for r, (dx, dy) in enumerate(DIRS):
        # 1/d(p) - 1/d(q) = -(n^T K^-1 (p - q)) / c with p - q = r
        v = -(n @ (Ki @ np.array([dx, dy, 0.0]))) / c / step
        exp = np.clip(np.sign(v) * np.floor(abs(v) + 0.5), -7, 7)
        got = dI[r, 2:-2, 2:-2, 0]
        assert np.mean(got == exp) > 0.999, (r, v, np.unique(got))
    assert np.array_equal(dI[2], -dI[3])
    assert np.all(dI[0] == 0)                     # plane constant along x: no jump
    z = orc.delta_i(np.zeros((4, 5), np.float32), nb[:4, :5], Ki, np.array([[0, 0, -1.0]]), [deltas])
    assert not z.any()


def _index_interp(deltas, iv):
    """Continuous index of inverse distances iv in a list of increasing
    distances, by numpy's piecewise-linear interpolation, extended linearly
    beyond the ends (independent of the oracle's scan)."""
    inv = 1.0 / np.asarray(deltas, np.float64)
    idx = np.arange(len(inv), dtype=np.float64)
    iv = np.asarray(iv, np.float64)
    j = np.interp(iv, inv[::-1], idx[::-1])
    lo = iv > inv[0]
    j = np.where(lo, (inv[0] - iv) / (inv[0] - inv[1]), j)
    hi = iv < inv[-1]
    G = len(inv)
    j = np.where(hi, G - 2 + (inv[-2] - iv) / (inv[-2] - inv[-1]), j)
    return j


def test_list_index_pins(orc):
    """The continuous plane index: exact at every plane, affine in inverse
    distance for a list uniform in it, and numpy's piecewise-linear
    interpolation (extended past the ends) for a list of varying spacing."""
    uni = orc.plane_list(20.0, 400.0, 64)
    step = (1 / 20 - 1 / 400) / 63
    for j in (0, 1, 17, 62, 63):
        assert abs(orc.list_index(uni, 1.0 / uni[j]) - j) < 1e-9
    rng = np.random.default_rng(9)
    for iv in rng.uniform(1 / 600, 1 / 15, 50):
        assert abs(orc.list_index(uni, iv) - (1 / 20 - iv) / step) < 1e-7
    geo = 15.0 * 1.07 ** np.arange(40) + np.cumsum(rng.random(40))
    ivs = rng.uniform(0.5 / geo[-1], 1.5 / geo[0], 200)
    got = np.array([orc.list_index(geo, iv) for iv in ivs])
    assert np.allclose(got, _index_interp(geo, ivs), atol=1e-9)


def test_level_list_pins(orc):
    """Finer-level lists: a list uniform in inverse distance stays uniform
    with the new count; whole fractional indices keep the coarse distances;
    other points lie on the piecewise-linear inverse-distance profile."""
    uni = orc.plane_list(20.0, 400.0, 32)
    for G in (64, 128, 32, 16):
        got = orc.level_list(uni, G)
        exp = orc.plane_list(20.0, 400.0, G)
        assert np.allclose(1 / got, 1 / exp, rtol=0, atol=1e-15), G
    rng = np.random.default_rng(5)
    geo = 12.0 * 1.1 ** np.arange(33) + np.cumsum(rng.random(33))
    fine = orc.level_list(geo, 129)      # 4x: every fourth plane is a coarse one
    assert np.array_equal(fine[::4], geo)
    u = np.arange(129) * 32 / 128
    exp = 1 / np.interp(u, np.arange(33), 1 / geo)
    assert np.allclose(fine, exp, rtol=1e-13)
    assert np.all(np.diff(fine) > 0)


def test_delta_i_on_an_analytic_plane_with_varying_plane_spacing(orc):
    """The same slanted plane with a list of varying spacing: the index jump
    toward each predecessor is the difference of the continuous indices
    (numpy's interpolation over the list) of the two points' inverse
    distances, rounded half away from zero and clamped to +-7."""
    K = np.array([[300.0, 0, 40], [0, 300.0, 30], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    n = np.array([0.0, 0.6, -0.8])
    c = 40.0
    d, _ = _plane_depth(Ki, n, c, 80, 60)
    geo = 30.0 * 1.0015 ** np.arange(512)
    nb = np.broadcast_to(n, (60, 80, 3)).astype(np.float32).copy()
    dI = orc.delta_i(d.astype(np.float32), nb, Ki, np.array([[0, 0, -1.0]]), [geo])
    DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]
    yy, xx = np.mgrid[0:60, 0:80]
    d32 = d.astype(np.float32).astype(np.float64)
    ip = 1.0 / d32
    nonzero = 0
    for r, (dx, dy) in enumerate(DIRS):
        # the predecessor's point on the seed's tangent plane (the plane itself)
        uq, vq = xx - dx + 0.5, yy - dy + 0.5
        ray_q = np.stack([uq, vq, np.ones_like(uq)], -1) @ Ki.T
        up, vp = xx + 0.5, yy + 0.5
        ray_p = np.stack([up, vp, np.ones_like(up)], -1) @ Ki.T
        dT = (n @ np.moveaxis(d32[..., None] * ray_p, -1, 0).reshape(3, -1)).reshape(60, 80) / (ray_q @ n)
        iq = 1.0 / dT
        v = _index_interp(geo, iq.ravel()).reshape(60, 80) - _index_interp(geo, ip.ravel()).reshape(60, 80)
        v = np.clip(v, -7, 7)
        exp = np.sign(v) * np.floor(np.abs(v) + 0.5)
        # rounding decisions within 1e-9 of a half are left out
        clear = np.abs(np.abs(v) - np.floor(np.abs(v)) - 0.5) > 1e-9
        got = dI[r, :, :, 0]
        assert np.array_equal(got[clear], exp[clear]), r
        nonzero += np.count_nonzero(exp)
    assert nonzero > 1000
