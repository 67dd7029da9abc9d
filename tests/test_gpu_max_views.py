"""Eight matching views, the most a bundle takes: census 5x5 (24 bits, so
eight views on one side still fit the 8-bit cost) and NCC 5x5 cost volumes
built from the images through the C ABI, against the oracle, for every kind
of left/right split (all left, all right, five and three), so a pixel's
per-view sums reach their largest values.  Ragged 83x45 frame (two tile
columns, two tile rows), 12 planes, random textures and near-identity
homographies with a projective part."""
import numpy as np
import pytest

from parity_util import assert_costs_from_images

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    import paper_2112_00821_amd as fm
    with fm.Handle() as h:
        yield h

N_VIEWS, H_IMG, W_IMG, G = 8, 45, 83, 12
SPLITS = {"all_left": [-1] * 8, "all_right": [1] * 8, "five_three": [-1, 1, -1, -1, 1, -1, 1, -1]}


def _inputs(seed):
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 256, (H_IMG, W_IMG)).astype(np.uint8)
    views = [rng.integers(0, 256, (H_IMG, W_IMG)).astype(np.uint8) for _ in range(N_VIEWS)]
    H = np.zeros((N_VIEWS, G, 3, 3))
    for k in range(N_VIEWS):
        for g in range(G):
            a, b, c, d = rng.normal(0, 0.02, 4)
            e, f = rng.normal(0, 2e-4, 2)
            H[k, g] = [[1 + a, b, 0.6 * g - k], [c, 1 + d, 0.3 * k], [e, f, 1.0]]
    return ref, views, H


@pytest.mark.parametrize("split", sorted(SPLITS))
def test_census_cost_eight_views(orc, hd, split):
    side = SPLITS[split]
    ref, views, H = _inputs(11)
    cw, ch = 5, 5   # 24 bits: with m = 8 views on one side a 9x7 cost would not fit 8 bits
    want = orc.cost_volume(orc.census(ref, cw, ch), views, side, cw, ch, [G], [G], H)
    ct = hd.stage_census(hd.upload(ref), cw, ch)
    got = hd.stage_cost(ct, [hd.upload(v) for v in views], side, cw, ch, [G], [G], H).numpy()
    assert_costs_from_images(got, want, f"census {split}")


@pytest.mark.parametrize("split", sorted(SPLITS))
def test_ncc_cost_eight_views(orc, hd, split):
    side = SPLITS[split]
    ref, views, H = _inputs(12)
    cw, ch = 5, 5
    want = orc.ncc_cost_volume(ref, views, side, cw, ch, [G], [G], H)
    got = hd.stage_cost_ncc(hd.upload(ref), [hd.upload(v) for v in views], side, cw, ch, [G], [G], H).numpy()
    assert_costs_from_images(got, want, f"ncc {split}")
