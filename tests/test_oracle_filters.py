"""Pins of the oracle's post-processing filters (Sec. on post-processing):
the DoG texture mask (Alg. 3) and the geometric consistency check by mutual
reprojection (Alg. 4)."""
import numpy as np
import pytest
from scipy import ndimage

import scenegen


def test_gauss_taps_normalised_symmetric(orc):
    t = orc.gauss_taps()
    assert t.shape == (7,)
    assert abs(t.sum() - 1.0) < 1e-15
    assert np.allclose(t, t[::-1], rtol=0, atol=0)
    # the Gaussian shape: ratio of neighbouring taps exp(-(2i+1)/(2 sigma^2))
    assert np.isclose(t[4] / t[3], np.exp(-1 / (2 * 1.4 ** 2)))


def test_dog_of_constant_and_ramp(orc):
    flat = np.full((20, 30), 90, np.uint8)
    assert np.max(np.abs(orc.dog(flat))) < 1e-12
    # a linear ramp is reproduced by a symmetric normalised kernel away from
    # the replicated border: DoG = 0 in the interior
    ramp = np.tile(np.arange(30, dtype=np.uint8) * 5, (20, 1))
    d = orc.dog(ramp)
    assert np.max(np.abs(d[:, 3:-3])) < 1e-9
    assert np.max(np.abs(d[:, :2])) > 0.5        # the clamped border bends it


@pytest.mark.parametrize("value,min_size", [(1, 7), (0, 21), (1, 3)])
def test_speckle_matches_connected_components(orc, value, min_size):
    """Speckle removal against scipy's 4-connected labelling."""
    rng = np.random.default_rng(min_size + value)
    m = (rng.random((40, 50)) < (0.35 if value == 1 else 0.65)).astype(np.uint8)
    got = orc.speckle(m, value, min_size)
    lab, n = ndimage.label(m == value)   # 4-connectivity by default
    sizes = ndimage.sum(np.ones_like(m), lab, index=np.arange(1, n + 1))
    small = np.isin(lab, np.arange(1, n + 1)[sizes < min_size])
    exp = m.copy()
    exp[small] = 1 - value
    assert np.array_equal(got, exp)


def test_dog_mask_closed_forms(orc):
    # flat image: no activation at all -> everything weakly textured
    assert not orc.dog_mask(np.full((40, 40), 120, np.uint8)).any()
    # strong texture everywhere: every pixel textured
    rng = np.random.default_rng(0)
    tex = rng.integers(0, 256, (40, 40)).astype(np.uint8)
    assert orc.dog_mask(tex).all()
    # a textured square on a flat background: the mask is the square grown by
    # the dilation and the smoothing footprint, never the far background
    img = np.full((60, 60), 100, np.uint8)
    img[20:40, 20:40] = tex[:20, :20]
    m = orc.dog_mask(img)
    assert m[25:35, 25:35].all()
    assert not m[:10].any() and not m[:, :10].any()


def test_dog_mask_matches_a_scipy_pipeline(orc):
    """The same pipeline assembled from library pieces (scipy convolution and
    labelling, double precision): identical masks on a rendered frame."""
    wl = scenegen.make_workload("config1")
    img = wl["ref"]["img"]
    t = orc.gauss_taps()
    sm = ndimage.correlate1d(img.astype(np.float64), t, axis=1, mode="nearest")
    sm = ndimage.correlate1d(sm, t, axis=0, mode="nearest")
    dog = img.astype(np.float64) - sm
    assert np.max(np.abs(dog - orc.dog(img))) < 1e-9
    on = (np.abs(dog) > 0.5).astype(np.uint8)
    # decisions within 1e-9 of the threshold could differ between summation
    # orders; the rendered frame has none
    assert np.min(np.abs(np.abs(dog) - 0.5)) > 1e-9

    def spk(m, v, k):
        lab, n = ndimage.label(m == v)
        sizes = ndimage.sum(np.ones_like(m), lab, index=np.arange(1, n + 1))
        out = m.copy()
        out[np.isin(lab, np.arange(1, n + 1)[sizes < k])] = 1 - v
        return out
    on = spk(on, 1, 7)
    on = ndimage.binary_dilation(on, structure=np.ones((3, 3))).astype(np.uint8)
    on = spk(on, 0, 21)
    assert np.array_equal(orc.dog_mask(img), on)


def _plane_depth(K, R, t, n, delta, w, h):
    """Depth map of the plane n.X + delta = 0 (world frame) seen from a camera
    x_cam = R x_world + t."""
    Ki = np.linalg.inv(K)
    u, v = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    ray = np.stack([u, v, np.ones_like(u)], -1) @ Ki.T          # camera coordinates, z = 1
    C = -R.T @ t
    dirw = ray @ R                                              # R^T ray
    s = -(n @ C + delta) / (dirw @ n)
    return (s * 1.0).astype(np.float32)                         # z of the ray point = s


def test_geo_consistency_on_exact_plane_maps(orc):
    """Depth maps of one world plane rendered exactly from five cameras: every
    pixel whose reprojection lands inside the neighbours is a hit; with all
    four neighbours in view the pixel is kept."""
    w, h = 64, 48
    K = np.array([[60.0, 0, 32], [0, 60.0, 24], [0, 0, 1]])
    n = np.array([0.0, 0.0, -1.0])
    Rs, ts = [], []
    for i, x in enumerate([-2.0, -1.0, 0.0, 1.0, 2.0]):
        Rs.append(np.eye(3))
        ts.append(np.array([-x, 0.0, 0.0]))
    deps = [_plane_depth(K, Rs[i], ts[i], n, 30.0, w, h) for i in range(5)]
    ref = 2
    nb = [i for i in range(5) if i != ref]
    Rr = [Rs[k] @ Rs[ref].T for k in nb]
    tr = [ts[k] - Rs[k] @ Rs[ref].T @ ts[ref] for k in nb]
    hits, keep = orc.geo_consistency(K, deps[ref], [deps[k] for k in nb], Rr, tr, 10.0, 3)
    # interior pixels (every neighbour sees them): four hits
    assert np.all(hits[:, 8:-8] == 4)
    assert keep[:, 8:-8].all()
    # a 2 m neighbour whose map reads a fifth of the true depth: reprojection
    # error f b |1/Z' - 1/Z| = 60 * 2 * (5/30 - 1/30) = 16 px > 10, a miss
    far = [j for j, k in enumerate(nb) if abs(k - ref) == 2]
    bad = [deps[k] * (0.2 if j == far[0] else 1.0) for j, k in enumerate(nb)]
    hits2, keep2 = orc.geo_consistency(K, deps[ref], bad, Rr, tr, 10.0, 3)
    assert np.all(hits2[:, 8:-8] == 3) and keep2[:, 8:-8].all()
    # both 2 m neighbours wrong: two hits, below the threshold, invalidated
    bad2 = [deps[k] * (0.2 if j in far else 1.0) for j, k in enumerate(nb)]
    hits3, keep3 = orc.geo_consistency(K, deps[ref], bad2, Rr, tr, 10.0, 3)
    assert np.all(hits3[:, 8:-8] == 2)
    assert not keep3[:, 8:-8].any()


def test_geo_consistency_error_closed_form(orc):
    """Fronto plane at depth Z, a neighbour translated by b along x whose map
    reads Z' everywhere: p goes to p - f b / Z in the neighbour and comes back
    at p - f b / Z + f b / Z', an error of f b |1/Z' - 1/Z|, checked on both
    sides of the threshold."""
    w, h = 40, 30
    f, b, Z = 50.0, 1.0, 20.0
    K = np.array([[f, 0, 20], [0, f, 15], [0, 0, 1]])
    dref = np.full((h, w), Z, np.float32)
    R = [np.eye(3)]
    t = [np.array([-b, 0.0, 0.0])]
    # p_k = p - f b / Z; lifted with Z' and mapped back: p' = p_k + f b / Z'
    # -> error = f b |1/Z' - 1/Z|
    for Zp, expect_hit in [(19.0, True), (10.0, True), (4.05, True), (3.95, False), (2.0, False)]:
        err = f * b * abs(1.0 / Zp - 1.0 / Z)
        hits, _ = orc.geo_consistency(K, dref, [np.full((h, w), Zp, np.float32)], R, t, 10.0, 1)
        inner = hits[:, 5:-5]
        assert np.all(inner == (1 if err < 10.0 else 0)), (Zp, err)
        assert (err < 10.0) == expect_hit
