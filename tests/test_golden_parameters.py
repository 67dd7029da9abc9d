"""The parameter values the paper prints (tests/golden/paper_parameters.json,
each with its passage) are the defaults of the oracle and of the library."""
import inspect
import json
import math
import os
import re

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = {v["name"]: v["value"] for v in json.load(open(os.path.join(HERE, "golden", "paper_parameters.json")))["values"]}


@pytest.fixture(scope="module")
def cfg():
    import paper_2112_00821_amd as fm
    return fm.default_config()


def test_library_defaults_are_the_printed_values(cfg):
    assert cfg.p2_alpha == GOLD["p2_alpha"] and cfg.p2_beta == GOLD["p2_beta"]
    assert cfg.normal_beta == GOLD["normal_beta"]
    assert cfg.conf_rho_deg == GOLD["conf_rho_deg"]
    assert cfg.median == 1   # the 5x5 median is on
    assert (cfg.census_w, cfg.census_h) == (GOLD["census_large_w"], GOLD["census_large_h"])
    assert cfg.p1 == GOLD["p1_census_9x7"]


def test_plane_cap_in_the_header():
    txt = open(os.path.join(HERE, "..", "include", "fassmvs.h")).read()
    m = re.search(r"#define FASSMVS_MAX_TOP_PLANES (\d+)", txt)
    assert m and int(m.group(1)) == GOLD["max_top_planes"]


def test_census_9x7_fills_62_of_64_bits(orc):
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (40, 50)).astype(np.uint8)
    cw, ch = GOLD["census_large_w"], GOLD["census_large_h"]
    ct = orc.census(img, cw, ch)
    nbits = cw * ch - 1
    assert nbits == 62 and nbits <= 64 < (cw * 9 - 1)   # 9x9 would need 80 bits
    assert int(ct.max()) < (1 << nbits) and int(ct.max()) >= (1 << (nbits - 1))


def test_p2_lut_takes_alpha_8_beta_10(orc):
    p1 = GOLD["p1_census_9x7"]
    lut = orc.p2_lut(p1, 1, 0, GOLD["p2_alpha"], GOLD["p2_beta"])
    for d in (0, 1, 10, 37, 255):
        want = math.floor(p1 * (1 + GOLD["p2_alpha"] * math.exp(-d / GOLD["p2_beta"])) + 0.5)
        assert lut[d] == want, (d, lut[d], want)
    assert lut[0] == 9 * p1


def test_pyramid_taps_are_the_sigma_1_gaussian():
    # the 3x3 sigma = 1 Gaussian on the 1/256 grid the pyramid uses
    g = np.exp(-np.arange(-1, 2) ** 2 / (2 * GOLD["pyramid_sigma"] ** 2))
    assert len(g) == GOLD["pyramid_kernel"]
    assert np.array_equal(np.round(256 * g / g.sum()).astype(int), [70, 116, 70])


def test_oracle_post_filter_defaults(orc):
    assert 2 * orc.DOG_RADIUS + 1 == GOLD["dog_kernel"]
    assert orc.DOG_THRESH == GOLD["dog_threshold"]
    assert (orc.DOG_MIN_ON, orc.DOG_MIN_OFF) == (GOLD["dog_min_on"], GOLD["dog_min_off"])
    sig = inspect.signature(orc.geo_consistency)
    assert sig.parameters["eta_r"].default == GOLD["geo_eta_r"]
    assert sig.parameters["eta_h"].default == GOLD["geo_eta_h"]


def test_library_geometric_filter_defaults():
    import paper_2112_00821_amd as fm
    sig = inspect.signature(fm.Handle.filter_geometric)
    assert sig.parameters["eta_r"].default == GOLD["geo_eta_r"]
    assert sig.parameters["eta_h"].default == GOLD["geo_eta_h"]


def test_ncc_penalty_and_scale(orc):
    import scenegen
    assert inspect.signature(scenegen.with_ncc).parameters["p1"].default == GOLD["p1_ncc"]
    flat = np.full((5, 5), 9, np.uint8)
    assert orc.ncc_window(flat, np.arange(25, dtype=np.float32).reshape(5, 5)) == GOLD["ncc_max_cost"]
