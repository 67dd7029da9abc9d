"""Oracle pins: cost volume, left/right combination, semi-global aggregation,
winner-takes-all and sub-plane refinement."""
import itertools

import numpy as np
import pytest

import scenegen


def _popcount(v):
    return np.vectorize(lambda x: bin(int(x)).count("1"))(v)


def _small_bundle(orc, name="config1"):
    wl = scenegen.make_workload(name)
    ref = wl["ref"]["img"]
    K = np.asarray(wl["K"])
    Ki, Kl = orc.kinv_level(K, 0)
    plan = orc.level_plan(wl, 0)
    rel = [orc.relative_pose(wl["ref"]["R"], wl["ref"]["t"], v["R"], v["t"]) for v in wl["views"]]
    H = np.array([[orc.homography(Kl, Ki, R, t, plan["fam_n"][0], d) for d in plan["deltas"][0]] for R, t in rel])
    return wl, ref, H, plan


def test_cost_volume_matches_per_sample_path(orc):
    wl, ref, H, plan = _small_bundle(orc)
    views = [v["img"] for v in wl["views"]]
    ct = orc.census(ref, 5, 5)
    S = orc.cost_volume(ct, views, wl["side"], 5, 5, plan["G"], plan["W"], H)
    rng = np.random.default_rng(0)
    h, w, D = S.shape
    for _ in range(200):
        x, y, g = rng.integers(0, w), rng.integers(0, h), rng.integers(0, D)
        assert S[y, x, g] == orc.cost_sample(ct, views, wl["side"], 5, 5, plan["G"], H, 0, g, x, y)
    for (x, y) in ((0, 0), (w - 1, h - 1), (0, h - 1), (w - 1, 0)):
        assert S[y, x, 5] == orc.cost_sample(ct, views, wl["side"], 5, 5, plan["G"], H, 0, 5, x, y)


def test_cost_volume_sum_and_lr_min(orc):
    """Multi-view cost = occlusion-robust minimum (Alg. 1) of the per-side sums
    of single-view Hamming costs; uneven subsets scale by m/|X|."""
    wl, ref, H, plan = _small_bundle(orc, "config2_small")
    # top level of the small config-2 scene: 4 views, 2 left + 2 right
    ct = orc.census(ref, 9, 7)
    views = [v["img"] for v in wl["views"]]
    G = [8]
    Hs = H[:, 10:18]
    single = [orc.cost_volume(ct, [views[k]], [-1], 9, 7, G, G, Hs[k:k + 1]).astype(int) for k in range(4)]
    S = orc.cost_volume(ct, views, [-1, -1, 1, 1], 9, 7, G, G, Hs).astype(int)
    assert np.array_equal(S, np.minimum(single[0] + single[1], single[2] + single[3]))
    S1 = orc.cost_volume(ct, views[:3], [-1, -1, -1], 9, 7, G, G, Hs[:3]).astype(int)
    assert np.array_equal(S1, single[0] + single[1] + single[2])
    S2 = orc.cost_volume(ct, views[:3], [-1, 1, 1], 9, 7, G, G, Hs[:3]).astype(int)
    assert np.array_equal(S2, np.minimum(2 * single[0], single[1] + single[2]))


def test_cost_zero_on_identical_view(orc):
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (20, 24)).astype(np.uint8)
    ct = orc.census(img, 5, 5)
    S = orc.cost_volume(ct, [img, img], [-1, 1], 5, 5, [1], [1], np.eye(3)[None, None].repeat(2, 0))
    assert S.max() == 0


def test_cost_volume_window_offsets(orc):
    """The dynamic cost volume stores, for each pixel, its window of the
    global plane list: entry i equals the full-volume entry offs + i."""
    wl, ref, H, plan = _small_bundle(orc)
    views = [v["img"] for v in wl["views"]]
    ct = orc.census(ref, 5, 5)
    full = orc.cost_volume(ct, views, wl["side"], 5, 5, [32], [32], H)
    rng = np.random.default_rng(2)
    offs = rng.integers(0, 32 - 8 + 1, (1,) + ref.shape).astype(np.int32)
    win = orc.cost_volume(ct, views, wl["side"], 5, 5, [32], [8], H, offs)
    yy, xx = np.mgrid[0:ref.shape[0], 0:ref.shape[1]]
    for i in range(8):
        assert np.array_equal(win[..., i], full[yy, xx, offs[0] + i])


# --------------------------------------------------------------------------
# semi-global aggregation
# --------------------------------------------------------------------------

def _brute_path(S, V):
    """min over all label sequences of sum S + sum V (1-pixel-wide image)."""
    n, D = S.shape
    best = None
    for seq in itertools.product(range(D), repeat=n):
        e = sum(S[t, seq[t]] for t in range(n)) + sum(V(t, seq[t], seq[t - 1]) for t in range(1, n))
        best = e if best is None else min(best, e)
    return best


@pytest.mark.parametrize("case", range(12))
def test_sgm_single_path_bruteforce(orc, case):
    """On a 1-pixel-wide image the downward path is exact dynamic
    programming: min_u L(last, u) plus the subtracted minima equals the
    brute-force minimum over all label sequences (Eq. sgm-path with
    Eq. sgm-smooth-fp / sgm-smooth-sn; windows and two families included)."""
    rng = np.random.default_rng(100 + case)
    n = int(rng.integers(2, 7))
    nf = 1 if case < 6 else 2
    Wf = [int(rng.integers(1, 4)) for _ in range(nf)]
    use_win = case % 2 == 1
    if use_win:
        Gf = [wv + int(rng.integers(0, 4)) for wv in Wf]
        offs = np.stack([rng.integers(0, g - wv + 1, (n, 1)) for g, wv in zip(Gf, Wf)]).astype(np.int32)
    else:
        Gf, offs = list(Wf), None
    D = sum(Wf)
    S = rng.integers(0, 40, (n, 1, D)).astype(np.uint8)
    p1 = int(rng.integers(0, 10))
    p2 = p1 + int(rng.integers(0, 30))
    ref = rng.integers(0, 256, (n, 1)).astype(np.uint8)
    lut = np.full(256, p2, np.int32)
    dI = np.zeros((8, n, 1, nf), np.int8)
    if case % 3 == 2:
        dI[2] = rng.integers(-2, 3, (n, 1, nf))
    foff = np.concatenate([[0], np.cumsum(Wf)])[:-1]

    def glob(t, u):
        f = int(np.searchsorted(foff, u, side="right") - 1)
        o = offs[f, t, 0] if offs is not None else 0
        return f, o + u - foff[f]

    def V(t, u, up):
        f, g = glob(t, u)
        fq, gq = glob(t - 1, up)
        if f != fq:
            return p2
        d = abs(g + dI[2, t, 0, f] - gq)
        return 0 if d == 0 else (p1 if d == 1 else p2)

    _, Lr = orc.sgm(S, Wf, p1, lut, ref, 4, offs=offs, dI=dI, want_sbar=False, want_lr=True)
    L = Lr[2, :, 0, :].astype(np.int64)                    # direction (0, 1)
    sub = sum(int(L[t - 1].min()) for t in range(1, n))
    assert int(L[-1].min()) + sub == _brute_path(S[:, 0, :].astype(np.int64), V)


def test_sgm_zero_penalties_is_wta(orc):
    rng = np.random.default_rng(3)
    S = rng.integers(0, 60, (9, 11, 6)).astype(np.uint8)
    ref = rng.integers(0, 256, (9, 11)).astype(np.uint8)
    for paths in (4, 8):
        Sbar, _ = orc.sgm(S, [6], 0, np.zeros(256, np.int32), ref, paths)
        assert np.array_equal(Sbar.astype(int), paths * S.astype(int))


def test_sgm_per_pixel_shift_invariance(orc):
    """Adding c to S(p, .) shifts S-bar(p, .) by n_paths * c and leaves every
    other pixel unchanged (normalised recursion, reading of Eq. sgm-path)."""
    rng = np.random.default_rng(4)
    S = rng.integers(0, 50, (7, 9, 5)).astype(np.uint8)
    ref = rng.integers(0, 256, (7, 9)).astype(np.uint8)
    lut = orc.p2_lut(8, 1, 0, 8.0, 10.0)
    Sbar, _ = orc.sgm(S, [5], 8, lut, ref, 8)
    S2 = S.copy()
    S2[3, 4] += 17
    Sbar2, _ = orc.sgm(S2, [5], 8, lut, ref, 8)
    diff = Sbar2.astype(int) - Sbar.astype(int)
    assert np.all(diff[3, 4] == 8 * 17)
    diff[3, 4] = 0
    assert np.all(diff == 0)


def test_sgm_mirror_and_transpose_invariance(orc):
    rng = np.random.default_rng(5)
    S = rng.integers(0, 50, (8, 10, 7)).astype(np.uint8)
    ref = rng.integers(0, 256, (8, 10)).astype(np.uint8)
    lut = orc.p2_lut(6, 1, 0, 8.0, 10.0)
    for paths in (4, 8):
        base, _ = orc.sgm(S, [7], 6, lut, ref, paths)
        fl, _ = orc.sgm(S[:, ::-1].copy(), [7], 6, lut, ref[:, ::-1].copy(), paths)
        assert np.array_equal(fl[:, ::-1], base)
        fv, _ = orc.sgm(S[::-1].copy(), [7], 6, lut, ref[::-1].copy(), paths)
        assert np.array_equal(fv[::-1], base)
        tr, _ = orc.sgm(S.transpose(1, 0, 2).copy(), [7], 6, lut, ref.T.copy(), paths)
        assert np.array_equal(tr.transpose(1, 0, 2), base)


def test_sgm_bound_and_zero_offsets(orc):
    rng = np.random.default_rng(6)
    S = rng.integers(0, 124, (10, 12, 16)).astype(np.uint8)
    ref = rng.integers(0, 256, (10, 12)).astype(np.uint8)
    lut = orc.p2_lut(48, 1, 0, 8.0, 10.0)
    Sbar, Lr = orc.sgm(S, [16], 48, lut, ref, 8, want_lr=True)
    assert Lr.max() <= 123 + lut.max()
    z, _ = orc.sgm(S, [16], 48, lut, ref, 8, dI=np.zeros((8, 10, 12, 1), np.int8))
    assert np.array_equal(z, Sbar)
    o, _ = orc.sgm(S, [16], 48, lut, ref, 8, offs=np.full((1, 10, 12), 5, np.int32))
    assert np.array_equal(o, Sbar)       # equal offsets everywhere: same transitions


def test_duplicate_family_keeps_wta(orc):
    rng = np.random.default_rng(7)
    S = rng.integers(0, 60, (6, 7, 5)).astype(np.uint8)
    ref = rng.integers(0, 256, (6, 7)).astype(np.uint8)
    lut = orc.p2_lut(8, 0, 40, 8.0, 10.0)
    one, _ = orc.sgm(S, [5], 8, lut, ref, 8)
    two, _ = orc.sgm(np.concatenate([S, S], -1), [5, 5], 8, lut, ref, 8)
    assert np.array_equal(two[..., :5], one) and np.array_equal(two[..., 5:], one)


# --------------------------------------------------------------------------
# winner-takes-all and refinement
# --------------------------------------------------------------------------

def test_wta_ties_and_refinement_vertex(orc):
    K = np.array([[100.0, 0, 8], [0, 100.0, 6], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    deltas = orc.plane_list(10.0, 50.0, 6)
    Sbar = np.zeros((1, 3, 6), np.uint16)
    Sbar[0, 0] = [50, 20, 20, 60, 70, 80]       # tie -> smaller index
    Sbar[0, 1] = [90, 70, 31, 40, 90, 99]
    Sbar[0, 2] = [5, 50, 60, 70, 80, 90]         # window end: no refinement
    label, fam, depth = orc.wta_refine(Sbar, [6], [6], np.array([[0, 0, -1.0]]), deltas, Ki)
    assert list(label[0]) == [1, 2, 0]
    assert depth[0, 2] == np.float32(deltas[0])
    # the refined depth is the vertex of the parabola through the three
    # (depth, cost) points, clamped to the neighbours' interval
    for x, i in ((0, 1), (1, 2)):
        d3 = deltas[i - 1:i + 2]
        c3 = Sbar[0, x, i - 1:i + 2].astype(float)
        a, b, _ = np.polyfit(d3, c3, 2)
        v = -b / (2 * a) if a > 0 else d3[1]
        v = min(max(v, d3[0]), d3[2])
        assert depth[0, x] == pytest.approx(v, rel=1e-6)


def test_refinement_matches_parabola_vertex(orc):
    K = np.array([[200.0, 0, 10], [0, 200.0, 10], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    deltas = orc.plane_list(20.0, 80.0, 9)
    rng = np.random.default_rng(8)
    for _ in range(40):
        i = int(rng.integers(1, 8))
        c = rng.integers(200, 400, 9)
        c[i] = rng.integers(0, 150)
        Sbar = c.astype(np.uint16)[None, None]
        label, _, depth = orc.wta_refine(Sbar, [9], [9], np.array([[0, 0, -1.0]]), deltas, Ki)
        assert label[0, 0] == i
        d3, c3 = deltas[i - 1:i + 2], c[i - 1:i + 2].astype(float)
        a, b, _ = np.polyfit(d3, c3, 2)
        assert a > 0
        assert depth[0, 0] == pytest.approx(min(max(-b / (2 * a), d3[0]), d3[2]), rel=1e-6)


# --------------------------------------------------------------------------
# path-gradient variant
# --------------------------------------------------------------------------

def _fronto_geom(orc, G, w):
    K = np.array([[300.0, 0, w / 2.0], [0, 300.0, 0.5], [0, 0, 1]])
    Ki, _ = orc.kinv_level(K, 0)
    deltas = orc.plane_list(20.0, 400.0, G)
    step = (1 / 20.0 - 1 / 400.0) / (G - 1)
    return dict(G=[G], fam_delta=deltas, fam_n=np.array([[0, 0, -1.0]]), Kinv=Ki, step=np.array([step]))


@pytest.mark.parametrize("seed", range(6))
def test_pg_fronto_offsets_continue_the_label_slope(orc, seed):
    """For fronto-parallel planes inverse depth is affine in the plane index,
    so the path-gradient extrapolation reduces exactly to continuing the
    previous step's label change: di_pg(p) = g(q2) - g(q) (clamped to 7)."""
    rng = np.random.default_rng(200 + seed)
    n, D = int(rng.integers(5, 30)), int(rng.integers(4, 20))
    S = rng.integers(0, 60, (1, n, D)).astype(np.uint8)
    p1 = int(rng.integers(1, 10))
    lut = np.full(256, p1 + int(rng.integers(0, 40)), np.int32)
    ref = rng.integers(0, 256, (1, n)).astype(np.uint8)
    geom = _fronto_geom(orc, D, n)
    _, Lr = orc.sgm(S, [D], p1, lut, ref, 4, want_sbar=False, want_lr=True, pg=geom)
    got = Lr[0, 0].astype(np.int64)            # direction (1, 0) along the row
    L = np.zeros((n, D), np.int64)
    L[0] = S[0, 0]
    arg = [int(np.argmin(L[0]))]
    for t in range(1, n):
        di = 0 if t < 2 else int(np.clip(arg[t - 2] - arg[t - 1], -7, 7))
        M = L[t - 1].min()
        for i in range(D):
            best = M + lut[0]
            for e in (-1, 0, 1):
                j = i + di + e
                if 0 <= j < D:
                    best = min(best, L[t - 1, j] + (0 if e == 0 else p1))
            L[t, i] = S[0, t, i] + best - M
        arg.append(int(np.argmin(L[t])))
    assert np.array_equal(got, L)


def test_pg_constant_winner_equals_plain(orc):
    rng = np.random.default_rng(9)
    S = rng.integers(40, 90, (9, 11, 12)).astype(np.uint8)
    S[..., 5] = 0
    ref = rng.integers(0, 256, (9, 11)).astype(np.uint8)
    lut = orc.p2_lut(8, 1, 0, 8.0, 10.0)
    geom = _fronto_geom(orc, 12, 11)
    a, _ = orc.sgm(S, [12], 8, lut, ref, 8)
    b, _ = orc.sgm(S, [12], 8, lut, ref, 8, pg=geom)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("fam_n", [(0.0, 0.0, -1.0), (0.0, 0.6, -0.8)])
def test_pg_locks_onto_an_analytic_slanted_plane(orc, fam_n):
    """A row of pixels seeing a plane whose plane index in the family's list
    rises by exactly 2 per pixel (inverse distance affine in x; for the
    slanted family n_x = 0 keeps n^T K^-1 p constant along the row), with
    the matching cost 0 on that index and 60 elsewhere: from the third
    pixel on, the path-gradient offset predicts the jump exactly
    (extrapolated inverse depth, di = -2), so the path cost at the plane's
    label is 0, where plain SGM pays P2 every step."""
    n_px, D, j0, p1, p2 = 14, 40, 3, 5, 30
    K = np.array([[200.0, 0.0, 7.0], [0.0, 200.0, 0.5], [0.0, 0.0, 1.0]])
    Ki, _ = orc.kinv_level(K, 0)
    nf = np.asarray(fam_n, np.float64)
    deltas = orc.plane_list(20.0, 400.0, D)
    iv = 1.0 / deltas
    step = (iv[0] - iv[-1]) / (D - 1)
    # rays of the row y = 0 and the family's n^T K^-1 p (constant along it)
    xs = np.arange(n_px) + 0.5
    rays = np.stack([xs, np.full(n_px, 0.5), np.ones(n_px)], -1) @ Ki.T
    cf = -(rays @ nf)
    assert np.allclose(cf, cf[0])
    S = np.full((1, n_px, D), 60, np.uint8)
    lab = j0 + 2 * np.arange(n_px)
    S[0, np.arange(n_px), lab] = 0
    lut = np.full(256, p2, np.int32)
    ref = np.zeros((1, n_px), np.uint8)
    geom = dict(G=[D], fam_delta=deltas, fam_n=nf[None], Kinv=Ki, step=np.array([step]))
    _, L_pg = orc.sgm(S, [D], p1, lut, ref, 4, want_sbar=False, want_lr=True, pg=geom)
    _, L_pi = orc.sgm(S, [D], p1, lut, ref, 4, want_sbar=False, want_lr=True)
    at_pg = L_pg[0, 0, np.arange(n_px), lab].astype(int)
    at_pi = L_pi[0, 0, np.arange(n_px), lab].astype(int)
    assert at_pg[0] == 0 and at_pg[1] == p2
    assert np.all(at_pg[2:] == 0), at_pg
    assert np.all(at_pi[1:] == p2), at_pi
    # the planes of the winning labels lie on one scene plane: their points'
    # inverse depth is affine along the row (what the extrapolation uses)
    inv_depth = cf / deltas[lab]
    assert np.allclose(np.diff(inv_depth, 2), 0, atol=1e-15)
