"""The C-ABI library loads and exports every symbol its public header
declares (no GPU needed; no compute call is made)."""
import ctypes as C

import pytest

import paper_2112_00821_amd as fm


def test_library_exports_every_header_symbol():
    L = fm.lib()
    names = fm.exported_symbols_in_header()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_config_matches_paper_settings():
    c = fm.default_config()
    assert (c.n_paths, c.census_w, c.census_h, c.p1) == (8, 9, 7, 24)
    assert c.p2_mode == 1 and c.p2_alpha == 8.0 and c.p2_beta == 10.0
    assert c.normal_beta == 10.0 and c.conf_rho_deg == 60.0 and c.median == 1


@pytest.mark.parametrize("field,value", [("n_paths", 6), ("census_w", 4), ("n_levels", 0), ("n_levels", 6),
                                         ("normal_radius", 9), ("conf_rho_deg", 95.0), ("window_labels", -1)])
def test_create_rejects_invalid_config_before_touching_the_device(field, value):
    c = fm.default_config()
    setattr(c, field, value)
    h = C.c_void_p()
    st = fm.lib().fassmvs_create(C.byref(c), C.byref(h))
    assert st == fm.EINVAL and not h.value
    assert fm.lib().fassmvs_last_error(None).decode()


def test_fixed_p2_below_p1_rejected():
    c = fm.default_config(p2_mode=0, p1=10, p2_fixed=5)
    h = C.c_void_p()
    assert fm.lib().fassmvs_create(C.byref(c), C.byref(h)) == fm.EINVAL


def test_unbuilt_census_window_is_unsupported():
    c = fm.default_config(census_w=11, census_h=5)
    h = C.c_void_p()
    assert fm.lib().fassmvs_create(C.byref(c), C.byref(h)) == fm.EUNSUPPORTED


def test_stage_names():
    names = [fm.lib().fassmvs_stage_name(i).decode() for i in range(fm.N_STAGES)]
    assert "sweep" in names and "sgm_dirs" in names and "sgm_wta" in names
    assert fm.lib().fassmvs_stage_name(99).decode() == ""
