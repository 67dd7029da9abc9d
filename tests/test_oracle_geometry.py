"""Oracle pins: camera geometry, plane sweep set-up, pyramid, warp, census.

Each check compares the oracle with something the paper or mathematics fixes
(closed forms, special cases, invariants), never with a retyped formula.
"""
import math

import numpy as np
import pytest


def _rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def _rand_K(rng):
    fx, fy = rng.uniform(100, 2000, 2)
    return np.array([[fx, rng.uniform(-2, 2), rng.uniform(50, 1000)],
                     [0.0, fy, rng.uniform(50, 800)], [0.0, 0.0, 1.0]])


def test_kinv_inverts_and_halves(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        K = _rand_K(rng)
        for l in range(4):
            Ki, Kl = orc.kinv_level(K, l)
            assert np.allclose(Kl @ Ki, np.eye(3), atol=1e-12)
            # the level intrinsics map a ray to 2^-l times the level-0 pixel-centre coordinates
            X = rng.normal(size=3) + np.array([0, 0, 10.0])
            p0 = K @ X
            pl = Kl @ X
            assert np.allclose(pl[:2] / pl[2], (p0[:2] / p0[2]) * 2.0 ** -l, rtol=1e-13)


def test_relative_pose_maps_ref_to_view(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        Rr, Rk = _rand_rot(rng), _rand_rot(rng)
        tr, tk = rng.normal(size=3) * 10, rng.normal(size=3) * 10
        R, t = orc.relative_pose(Rr, tr, Rk, tk)
        Xw = rng.normal(size=3) * 30
        assert np.allclose(R @ (Rr @ Xw + tr) + t, Rk @ Xw + tk, atol=1e-10)


def test_homography_closed_form(orc):
    """Points on n^T X + delta = 0 seen in the reference project into view k
    exactly where H maps their reference pixel (Eq. homography)."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        K = _rand_K(rng)
        Ki, Kl = orc.kinv_level(K, 0)
        R = _rand_rot(rng) if rng.random() < 0.5 else np.eye(3)
        t = rng.normal(size=3)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        if n[2] > 0:
            n = -n
        delta = rng.uniform(5, 100)
        H = orc.homography(Kl, Ki, R, t, n, delta)
        for _ in range(5):
            ray = Ki @ np.array([rng.uniform(0, 1000), rng.uniform(0, 800), 1.0])
            den = n @ ray
            if den >= -1e-3:
                continue
            X = ray * (-delta / den)
            assert abs(n @ X + delta) < 1e-9 * delta
            pr = K @ X
            pk = K @ (R @ X + t)
            hp = H @ pr
            assert np.allclose(hp / hp[2], pk / pk[2], rtol=1e-11, atol=1e-9)
    K = _rand_K(rng)
    Ki, Kl = orc.kinv_level(K, 0)
    assert np.allclose(orc.homography(Kl, Ki, np.eye(3), np.zeros(3), [0, 0, -1.0], 20.0), np.eye(3), atol=1e-12)


def test_depth_on_plane(orc):
    rng = np.random.default_rng(3)
    K = _rand_K(rng)
    Ki, _ = orc.kinv_level(K, 0)
    for _ in range(50):
        x, y = rng.integers(0, 900, 2)
        delta = rng.uniform(1, 500)
        # fronto-parallel sweep: depth equals the plane distance
        assert orc.depth_on_plane(Ki, [0, 0, -1.0], delta, x, y) == pytest.approx(delta, rel=1e-15)
        n = rng.normal(size=3)
        n[2] = -abs(n[2]) - 0.5
        n /= np.linalg.norm(n)
        d = orc.depth_on_plane(Ki, n, delta, x, y)
        if d > 0:
            X = d * (Ki @ np.array([x + 0.5, y + 0.5, 1.0]))
            assert abs(n @ X + delta) < 1e-9 * delta
    # a ray that does not meet the plane in front of the camera is invalid
    assert orc.depth_on_plane(Ki, [0, 0, 1.0], 10.0, 3, 3) == 0.0


def test_plane_list_inverse_uniform(orc):
    d = orc.plane_list(30.0, 120.0, 32)
    assert d[0] == pytest.approx(30.0, rel=1e-15)
    assert d[-1] == pytest.approx(120.0, rel=1e-13)
    inv = 1.0 / d
    assert np.allclose(np.diff(inv), (1 / 120 - 1 / 30) / 31, rtol=1e-9)
    assert np.all(np.diff(d) > 0)


def test_p2_lut_shape(orc):
    """Eq. p2-grad: P2(0) = P1 (1 + alpha); P2 -> P1 for large gradients;
    decreasing; exp semigroup: (P2(2a)-P1) = (P2(a)-P1)^2 / (P1 alpha)."""
    p1 = 10000
    lut = orc.p2_lut(p1, 1, 0, 8.0, 10.0).astype(np.int64)
    assert lut[0] == p1 * 9
    assert np.all(np.diff(lut) <= 0)
    assert lut[255] == p1
    for a in (3, 5, 10, 20):
        lhs = lut[2 * a] - p1
        rhs = (lut[a] - p1) ** 2 / (p1 * 8.0)
        assert abs(lhs - rhs) <= 1.0 + 2 * (lut[a] - p1) / (p1 * 8.0)
    assert np.all(orc.p2_lut(48, 0, 64, 8.0, 10.0) == 64)


def test_pyramid_constant_ramp_impulse(orc):
    img = np.full((13, 17), 77, np.uint8)
    out = orc.pyr_down(img)
    assert out.shape == (6, 8) and np.all(out == 77)
    # a linear ramp survives the symmetric blur; the 2x2 mean samples it at
    # the level-1 pixel centre x = 2u + 0.5 (level-0 coordinates of the centre
    # of the block), which is what halving fx, cx requires
    ramp = np.tile((2 * np.arange(64)).astype(np.uint8), (8, 1))
    out = orc.pyr_down(ramp)
    u = np.arange(32)
    assert np.all(out[:, 1:-1] == (4 * u + 1)[1:-1])
    # impulse: the 3x3 sigma=1 Gaussian (paper) within quantisation error
    imp = np.zeros((16, 16), np.uint8)
    imp[8, 8] = 255
    out = orc.pyr_down(imp).astype(float)
    g = np.exp(-np.arange(-1, 2) ** 2 / 2.0)
    g /= g.sum()
    k = 255 * np.outer(g, g)
    blur = np.zeros((16, 16))
    blur[7:10, 7:10] = k
    ref = blur.reshape(8, 2, 8, 2).mean(axis=(1, 3))
    assert np.max(np.abs(out - ref)) <= 1.5
    assert abs(out.sum() * 4 - 255) <= 8


def test_pyramid_sizes(orc):
    for w, h in ((2, 2), (3, 5), (333, 187)):
        assert orc.pyr_down(np.zeros((h, w), np.uint8)).shape == (h // 2, w // 2)


def test_warp_identity_translation_halfpixel(orc):
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, (20, 30)).astype(np.uint8)
    out = orc.warp(img, np.eye(3), 30, 20)
    assert np.array_equal(out, img.astype(np.float32))
    T = np.array([[1, 0, 3.0], [0, 1, -2.0], [0, 0, 1]])
    out = orc.warp(img, T, 30, 20)
    yy, xx = np.mgrid[0:20, 0:30]
    exp = img[np.clip(yy - 2, 0, 19), np.clip(xx + 3, 0, 29)]
    assert np.array_equal(out, exp.astype(np.float32))
    Th = np.array([[1, 0, 0.5], [0, 1, 0.0], [0, 0, 1]])
    out = orc.warp(img, Th, 29, 20)
    assert np.array_equal(out, 0.5 * img[:, :29].astype(np.float32) + 0.5 * img[:, 1:30].astype(np.float32))
    # projective scaling of the homogeneous coordinate changes nothing
    assert np.array_equal(orc.warp(img, 3.7 * T, 30, 20), orc.warp(img, T, 30, 20))


def test_warp_reproduces_affine_ramp(orc):
    """Bilinear interpolation is exact on a linear intensity ramp."""
    xx, yy = np.meshgrid(np.arange(64), np.arange(48))
    img = (2 * xx + yy).astype(np.uint8)
    rng = np.random.default_rng(5)
    for _ in range(5):
        a = rng.uniform(-0.2, 0.2)
        A = np.array([[math.cos(a) * 0.9, -math.sin(a), 20.0], [math.sin(a), math.cos(a) * 0.9, 15.0], [0, 0, 1]])
        out = orc.warp(img, A, 20, 20)
        q = np.stack(np.meshgrid(np.arange(20) + 0.5, np.arange(20) + 0.5), -1)
        s = q @ A[:2, :2].T + A[:2, 2] - 0.5
        exp = 2 * s[..., 0] + s[..., 1]
        inside = (s[..., 0] >= 0) & (s[..., 0] <= 63) & (s[..., 1] >= 0) & (s[..., 1] <= 47)
        assert inside.mean() > 0.9
        assert np.max(np.abs(out[inside] - exp[inside])) < 1e-3


def test_warp_behind_camera_and_far_outside(orc):
    img = np.arange(12, dtype=np.uint8).reshape(3, 4) * 10
    Hb = np.array([[1, 0, 0], [0, 1, 0], [0, 0, -1.0]])
    assert np.all(orc.warp(img, Hb, 4, 3) == img[0, 0])
    Hf = np.array([[1, 0, 1e9], [0, 1, -1e9], [0, 0, 1.0]])
    assert np.all(orc.warp(img, Hf, 4, 3) == img[0, 3])


def test_census_closed_forms(orc):
    # values increase in row-major order: every neighbour before the centre is
    # smaller, so the word is (2^12 - 1) << 12 for 5x5 with MSB-first order
    img = (np.arange(10 * 10).reshape(10, 10)).astype(np.float32)
    ct = orc.census(img, 5, 5)
    assert int(ct[5, 5]) == 0xFFF000
    ct = orc.census(-img, 5, 5)
    assert int(ct[5, 5]) == 0x000FFF
    ct = orc.census(img, 9, 7)
    assert int(ct[5, 5]) == ((1 << 31) - 1) << 31
    assert orc.census(np.full((6, 9), 3.0, np.float32), 9, 7).max() == 0
    # replicate border: at (0,0) the rows above clamp onto row 0, so only the
    # positions that fall on row 0 left of the centre (clamped to the centre)
    # compare equal -> the word is zero for the increasing image
    assert int(orc.census(img, 5, 5)[0, 0]) == 0
    # uint8 and float inputs agree (k/1 monotone)
    u8 = np.random.default_rng(6).integers(0, 256, (12, 15)).astype(np.uint8)
    assert np.array_equal(orc.census(u8, 9, 7), orc.census(u8.astype(np.float32), 9, 7))


def test_census_hamming_metric(orc):
    rng = np.random.default_rng(7)
    a = rng.random((16, 16)).astype(np.float32)
    b = rng.random((16, 16)).astype(np.float32)
    c = rng.random((16, 16)).astype(np.float32)
    ca, cb, cc = (orc.census(x, 9, 7) for x in (a, b, c))
    pc = np.vectorize(lambda v: bin(int(v)).count("1"))
    dab, dbc, dac = pc(ca ^ cb), pc(cb ^ cc), pc(ca ^ cc)
    assert np.all(dac <= dab + dbc)
    assert np.all(pc(ca ^ ca) == 0)
    assert np.all(dab <= 62) and np.all(pc(ca) <= 62)
    # inverted intensities flip every bit that is not a tie
    ci = orc.census(-a, 9, 7)
    assert np.all(pc(ca ^ ci)[3:-3, 4:-4] == 62)


def _bilinear_f64(img, H, rw, rh):
    """Plain float64 bilinear clamp-to-edge warp written with numpy (no
    fused operations, no float32 rounding): the value at reference pixel q is
    the view sampled at H (q + 0.5) / hz - 0.5; a point behind the view's
    focal plane reads the top-left pixel."""
    h, w = img.shape
    I = img.astype(np.float64)
    yy, xx = np.mgrid[0:rh, 0:rw]
    q = np.stack([xx + 0.5, yy + 0.5, np.ones_like(xx, dtype=np.float64)], -1)
    p = q @ np.asarray(H, np.float64).T
    front = p[..., 2] > 1e-300
    with np.errstate(divide="ignore", invalid="ignore"):
        sx = np.where(front, p[..., 0] / p[..., 2], 0.0) - 0.5
        sy = np.where(front, p[..., 1] / p[..., 2], 0.0) - 0.5
    sx = np.clip(sx, -1.0, float(w))
    sy = np.clip(sy, -1.0, float(h))
    x0 = np.floor(sx)
    y0 = np.floor(sy)
    ax, ay = sx - x0, sy - y0
    x0 = x0.astype(int)
    y0 = y0.astype(int)
    xa, xb = np.clip(x0, 0, w - 1), np.clip(x0 + 1, 0, w - 1)
    ya, yb = np.clip(y0, 0, h - 1), np.clip(y0 + 1, 0, h - 1)
    top = I[ya, xa] * (1 - ax) + I[ya, xb] * ax
    bot = I[yb, xa] * (1 - ax) + I[yb, xb] * ax
    return top * (1 - ay) + bot * ay


@pytest.mark.parametrize("seed", range(8))
def test_warp_within_1e4_of_float64_bilinear(orc, seed):
    """The oracle's fixed warp (double coordinates, float interpolation)
    stays within 1e-4 (on the [0, 1] intensity scale) of a plain float64
    bilinear warp, on random images and random projective homographies
    that shrink, stretch, shear and move the view partly outside the
    image."""
    rng = np.random.default_rng(300 + seed)
    h, w = int(rng.integers(20, 90)), int(rng.integers(20, 120))
    img = rng.integers(0, 256, (h, w)).astype(np.uint8)
    A = np.eye(3)
    A[:2, :2] += rng.normal(0, 0.25, (2, 2))
    A[:2, 2] = rng.uniform(-0.3, 0.3, 2) * [w, h]
    A[2, :2] = rng.normal(0, 2e-3, 2)
    got = orc.warp(img, A, w, h)
    exp = _bilinear_f64(img, A, w, h)
    assert np.max(np.abs(got - exp)) / 255.0 <= 1e-4, np.max(np.abs(got - exp)) / 255.0


def test_warp_float64_behind_and_far_outside(orc):
    """Points behind the view and far outside: the same value as the float64
    definition (border pixels)."""
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (30, 40)).astype(np.uint8)
    for H in (np.diag([1.0, 1.0, -1.0]), np.array([[1, 0, 1e9], [0, 1, -1e9], [0, 0, 1.0]]),
              np.array([[1, 0, -1e7], [0, 1, 1e7], [0, 0, 1.0]]),
              np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.02, 0.0, -0.3]])):
        got = orc.warp(img, H, 40, 30)
        exp = _bilinear_f64(img, H, 40, 30)
        assert np.max(np.abs(got - exp)) / 255.0 <= 1e-4
