"""The library's host-side plane-set functions (bounding planes and the
cross-ratio list) against the oracle's.  Host code only: no GPU needed."""
import numpy as np
import pytest

import paper_2112_00821_amd as fm
import scenegen

K = np.array([[800.0, 0, 480], [0, 800.0, 270], [0, 0, 1]])


@pytest.mark.parametrize("n", [[0, 0, -1.0], [0, -np.sin(0.6), -np.cos(0.6)], [0.2, -0.3, -0.93]])
def test_bounding_planes_library_equals_oracle(orc, n):
    n = np.asarray(n) / np.linalg.norm(n)
    a = fm.bounding_planes(K, 960, 540, n, 15.0, 300.0)
    b = orc.bounding_planes(K, 960, 540, n, 15.0, 300.0)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", range(5))
def test_cross_ratio_library_equals_oracle(orc, case):
    rng = np.random.default_rng(case)
    a = rng.normal(0, 0.03, 3)
    Rx = np.array([[1, 0, 0], [0, np.cos(a[0]), -np.sin(a[0])], [0, np.sin(a[0]), np.cos(a[0])]])
    Ry = np.array([[np.cos(a[1]), 0, np.sin(a[1])], [0, 1, 0], [-np.sin(a[1]), 0, np.cos(a[1])]])
    R = Rx @ Ry
    t = rng.normal(0, 1.5, 3)
    t[2] *= 0.3
    n = np.array([0.0, -np.sin(0.3 * case), -np.cos(0.3 * case)])
    lo, hi = orc.bounding_planes(K, 960, 540, n, 20.0, 400.0)
    try:
        exp = orc.cross_ratio_planes(K, 960, 540, R, t, n, lo, hi)
    except ValueError:
        # degenerate for the oracle (camera behind the nearest plane): the
        # library must refuse it the same way
        with pytest.raises(fm.FassmvsError) as e:
            fm.cross_ratio_planes(K, 960, 540, R, t, n, lo, hi)
        assert e.value.status == fm.EINVAL
        return
    got = fm.cross_ratio_planes(K, 960, 540, R, t, n, lo, hi)
    assert len(got) == len(exp)
    assert np.allclose(got, exp, rtol=1e-12, atol=0)


def test_cross_ratio_capacity_and_errors():
    t = np.array([-20.0, 0, 0])
    with pytest.raises(fm.FassmvsError) as e:
        fm.cross_ratio_planes(K, 960, 540, np.eye(3), t, [0, 0, -1.0], 20.0, 400.0, max_planes=256)
    assert e.value.status == fm.EUNSUPPORTED
    with pytest.raises(fm.FassmvsError) as e:
        fm.cross_ratio_planes(K, 960, 540, np.eye(3), np.array([0, 0, -30.0]), [0, 0, -1.0], 20.0, 400.0)
    assert e.value.status == fm.EINVAL


def test_family_count_zero_uses_cross_ratio_length(orc):
    wl = scenegen.make_workload("config1")
    fam = dict(wl["families"][0], count=0)
    c = orc.family_count(dict(wl, families=[fam]), fam)
    assert 2 <= c <= 256
    K1, _ = orc.kinv_level(np.asarray(wl["K"]), 0)
    R, t = orc.relative_pose(wl["ref"]["R"], wl["ref"]["t"], wl["views"][0]["R"], wl["views"][0]["t"])
    assert c == len(orc.cross_ratio_planes(np.asarray(wl["K"]), wl["width"], wl["height"], R, t, fam["n"],
                                           fam["delta_min"], fam["delta_max"])) or c >= 2
