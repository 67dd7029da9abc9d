"""Pins of the oracle's NCC matching cost (negated, truncated and scaled
normalised cross-correlation; the similarity-measure section of the paper):
identity and affine-invariance give cost 0, anti-correlation and flat
windows the truncated maximum 255, and random windows agree with the
textbook correlation coefficient computed independently (two-pass, centred,
numpy) to within the rounding of the final scaling."""
import numpy as np
import pytest

import scenegen


def _ident_H(n_views, G):
    H = np.zeros((n_views, G, 3, 3))
    H[:, :] = np.eye(3)
    return H


@pytest.mark.parametrize("cw,ch", [(5, 5), (9, 9), (3, 3), (7, 5)])
def test_ncc_window_against_textbook_correlation(orc, cw, ch):
    rng = np.random.default_rng(cw * 10 + ch)
    for trial in range(300):
        a = rng.integers(0, 256, (ch, cw)).astype(np.uint8)
        b = (rng.random((ch, cw)) * 255).astype(np.float32)
        if trial % 3 == 0:          # strongly correlated windows
            b = np.clip(a * 0.7 + 30 + rng.normal(0, 5, (ch, cw)), 0, 255).astype(np.float32)
        if trial % 3 == 1:          # anti-correlated windows
            b = np.clip(255 - a * 0.9 + rng.normal(0, 5, (ch, cw)), 0, 255).astype(np.float32)
        av = a.astype(np.float64).ravel() - a.mean()
        bv = b.astype(np.float64).ravel() - b.astype(np.float64).mean()
        rho = float(av @ bv / np.sqrt((av @ av) * (bv @ bv)))
        exp = np.floor(255 * min(1.0, 1.0 - rho) + 0.5)
        got = orc.ncc_window(a, b)
        assert abs(got - exp) <= 1, (trial, got, exp, rho)


def test_ncc_window_closed_forms(orc):
    rng = np.random.default_rng(3)
    a = rng.integers(0, 128, (5, 5)).astype(np.uint8)
    assert orc.ncc_window(a, a.astype(np.float32)) == 0                 # identical
    assert orc.ncc_window(a, (2.0 * a + 1).astype(np.float32)) == 0     # gain and offset (exact in float)
    assert orc.ncc_window(a, (255.0 - a).astype(np.float32)) == 255     # anti-correlated: truncated
    flat = np.full((5, 5), 77, np.uint8)
    assert orc.ncc_window(flat, a.astype(np.float32)) == 255            # flat reference window
    assert orc.ncc_window(a, np.full((5, 5), 3.25, np.float32)) == 255  # flat warped window
    # uncorrelated by construction: rho = 0 -> 255 (cost of "1 - rho" truncated at 1)
    x = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], np.uint8) * 100
    y = np.array([[1, 1, 1], [0, 0, 0], [1, 1, 1]], np.float32) * 50
    assert orc.ncc_window(x, y) == 255


def test_ncc_cost_volume_identity_and_affine_views(orc):
    """Views that are the reference itself, or an exact affine intensity
    map of it, under the identity homography: every textured pixel costs 0
    for every label."""
    wl = scenegen.make_workload("config1")
    ref = wl["ref"]["img"]
    h, w = ref.shape
    img = (ref // 2).astype(np.uint8)                  # values <= 127
    aff = (2 * img.astype(np.int32) + 1).astype(np.uint8)
    G = 4
    S = orc.ncc_cost_volume(img, [img, aff], [-1, 1], 5, 5, [G], [G], _ident_H(2, G))
    # textured windows: zero cost; a flat window costs 255
    var = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            win = img[max(0, y - 2):y + 3, max(0, x - 2):x + 3]
            var[y, x] = win.std()
    tex = var > 2
    assert np.all(S[tex] == 0)


def test_ncc_combine_is_subset_mean(orc):
    """S = min over the non-empty subsets of the mean cost: one left view
    identical to the reference (cost 0) and two right views, one identical
    and one negated (costs 0 and 255): S = min(0, floor(255/2)) = 0; with
    only the right subset S = 127."""
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, (12, 14)).astype(np.uint8)
    neg = (255 - img).astype(np.uint8)
    H3 = _ident_H(3, 2)
    S = orc.ncc_cost_volume(img, [img, img, neg], [-1, 1, 1], 5, 5, [2], [2], H3)
    assert np.all(S == 0)
    H2 = _ident_H(2, 2)
    S2 = orc.ncc_cost_volume(img, [img, neg], [1, 1], 5, 5, [2], [2], H2)
    assert np.all(S2 == 127)


def test_ncc_cost_pixels_match_volume(orc):
    wl = scenegen.make_workload("config1")
    p = wl["params"]
    Ki, Kl = orc.kinv_level(np.asarray(wl["K"]), 0)
    plan = orc.level_plan(wl, 0)
    rel = [orc.relative_pose(wl["ref"]["R"], wl["ref"]["t"], v["R"], v["t"]) for v in wl["views"]]
    H = np.zeros((len(rel), plan["G"][0], 3, 3))
    for k, (R, t) in enumerate(rel):
        for j, dv in enumerate(plan["deltas"][0]):
            H[k, j] = orc.homography(Kl, Ki, R, t, plan["fam_n"][0], dv)
    views = [v["img"] for v in wl["views"]]
    S = orc.ncc_cost_volume(wl["ref"]["img"], views, wl["side"], 5, 5, plan["G"], plan["W"], H)
    xy = np.array([[0, 0], [159, 119], [80, 60], [3, 117], [150, 2]], np.int32)
    got = orc.ncc_cost_pixels(wl["ref"]["img"], views, wl["side"], 5, 5, plan["G"], plan["W"], H, xy)
    assert np.array_equal(got, S[xy[:, 1], xy[:, 0]])


def test_ncc_pipeline_recovers_ground_truth(orc):
    """The nadir scene with ground and roofs exactly on sweep planes, no
    noise: with the NCC cost the winner is the true plane on textured pixels
    away from depth edges, borders and occlusions."""
    from test_oracle_pipeline import _far_from_edges, _visible_in_views
    wl = scenegen.make_workload("nadir_planar")
    wl = dict(wl, params=dict(wl["params"], cost="ncc", census_w=5, census_h=5, p1=20, p2_fixed=60))
    out = orc.run_frame(wl, keep=True)
    lv = out["levels"][0]
    gt = wl["gt"]["depth"]
    deltas = np.asarray(wl["gt_plane_delta"])
    gt_idx = np.argmin(np.abs(gt[..., None] - deltas), axis=-1)
    on_plane = np.min(np.abs(gt[..., None] - deltas), axis=-1) < 1e-6 * gt
    mask = on_plane & _far_from_edges(gt, 3) & _visible_in_views(wl)
    assert mask.mean() > 0.5
    agree = lv["label"][mask] == gt_idx[mask]
    assert agree.mean() >= 0.995, agree.mean()
