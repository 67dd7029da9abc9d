"""Stage-by-stage parity of the gfx950 kernels with the CPU oracle.

Integer stages (pyramid, census, cost volume, path costs, aggregate, WTA,
window offsets, surface-normal offsets, median) must be bit-exact; the warp
is held to |diff| <= 1e-4 on the [0, 1] scale (and is bit-exact in practice:
coordinates are computed in double on both sides, the kernel's reciprocal
within an ulp of the oracle's); refined depth to 1e-6 relative (double
arithmetic on both sides); normals, smoothed normals and confidence
bit-exact.  Every call goes through the C ABI."""
import numpy as np
import pytest

import scenegen
from parity_util import assert_costs_from_images, assert_warp_close, first_mismatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    import paper_2112_00821_amd as fm
    return fm


@pytest.fixture(scope="module")
def hd(fm):
    with fm.Handle() as h:
        yield h


def _setup(orc, name, level=0):
    wl = scenegen.make_workload(name)
    out = orc.run_frame(wl, keep=True)
    return wl, out


@pytest.mark.parametrize("shape", [(120, 160), (187, 333), (9, 17), (2, 2)])
def test_pyramid_bit_exact(orc, hd, shape):
    rng = np.random.default_rng(shape[0])
    img = rng.integers(0, 256, shape).astype(np.uint8)
    got = hd.stage_pyr_down(hd.upload(img)).numpy()
    assert np.array_equal(got, orc.pyr_down(img))


@pytest.mark.parametrize("cw,ch", [(5, 5), (9, 7), (3, 3)])
@pytest.mark.parametrize("shape", [(120, 160), (37, 71)])
def test_census_bit_exact(orc, hd, cw, ch, shape):
    rng = np.random.default_rng(cw * 100 + shape[1])
    img = rng.integers(0, 256, shape).astype(np.uint8)
    img[5:15, 5:15] = 77                       # ties
    got = hd.stage_census(hd.upload(img), cw, ch).numpy()
    assert np.array_equal(got, orc.census(img, cw, ch))


def test_warp_matches_oracle(orc, hd):
    wl = scenegen.make_workload("config1")
    K = np.asarray(wl["K"])
    Ki, Kl = orc.kinv_level(K, 0)
    R, t = orc.relative_pose(wl["ref"]["R"], wl["ref"]["t"], wl["views"][0]["R"], wl["views"][0]["t"])
    src = wl["views"][0]["img"]
    dsrc = hd.upload(src)
    for delta in (30.0, 47.3, 120.0, 1e4):
        for n in ([0, 0, -1.0], [0.2, -0.3, -0.932737905]):
            n = np.asarray(n) / np.linalg.norm(n)
            H = orc.homography(Kl, Ki, R, t, n, delta)
            got = hd.stage_warp(dsrc, H, 160, 120).numpy()
            exp = orc.warp(src, H, 160, 120)
            assert_warp_close(got, exp, f"delta {delta}")
    # random homographies near the identity: every fractional position
    rng = np.random.default_rng(11)
    for _ in range(6):
        H = np.eye(3) + rng.normal(0, 0.01, (3, 3)) * np.array([[1, 1, 300], [1, 1, 300], [1e-4, 1e-4, 1]])
        assert_warp_close(hd.stage_warp(dsrc, H, 160, 120).numpy(), orc.warp(src, H, 160, 120), "random")
    # behind the camera and far outside: the border rules give the same pixels
    for H in (np.diag([1.0, 1.0, -1.0]), np.array([[1, 0, 1e9], [0, 1, -1e9], [0, 0, 1.0]])):
        assert np.array_equal(hd.stage_warp(dsrc, H, 160, 120).numpy(), orc.warp(src, H, 160, 120))


def _level_inputs(orc, wl, level):
    K = np.asarray(wl["K"])
    Ki, Kl = orc.kinv_level(K, level)
    plan = orc.level_plan(wl, level)
    rel = [orc.relative_pose(wl["ref"]["R"], wl["ref"]["t"], v["R"], v["t"]) for v in wl["views"]]
    sumG = sum(plan["G"])
    H = np.zeros((len(rel), sumG, 3, 3))
    for k, (R, t) in enumerate(rel):
        g0 = 0
        for f, dl in enumerate(plan["deltas"]):
            for j, dv in enumerate(dl):
                H[k, g0 + j] = orc.homography(Kl, Ki, R, t, plan["fam_n"][f], dv)
            g0 += len(dl)
    return Ki, Kl, plan, H


@pytest.mark.parametrize("name", ["config1", "config2_small"])
def test_cost_from_oracle_warps_bit_exact(orc, hd, name):
    """Census, Hamming and the left/right minimum are bit-exact when the
    kernel is fed the oracle's warped images."""
    wl = scenegen.make_workload(name)
    p = wl["params"]
    level = p["n_levels"] - 1
    out = orc.run_frame(wl, keep=True, levels_only=level)
    lv = out["levels"][level]
    Ki, Kl, plan, H = _level_inputs(orc, wl, level)
    views = [pv[level] for pv in out["pyr_views"]]
    h, w = lv["img"].shape
    warped = np.zeros((len(views), sum(plan["G"]), h, w), np.float32)
    for k in range(len(views)):
        for g in range(sum(plan["G"])):
            warped[k, g] = orc.warp(views[k], H[k, g], w, h)
    ct = hd.upload(lv["ct"])
    got = hd.stage_cost(ct, None, wl["side"], p["census_w"], p["census_h"], plan["G"], plan["W"], H,
                        warped=hd.upload(warped)).numpy()
    assert np.array_equal(got, lv["S"])


@pytest.mark.parametrize("name", ["config1", "config2_small", "config2_ragged", "config3_small"])
@pytest.mark.parametrize("rows", ["4", "8"])
def test_cost_volume_from_images(orc, hd, monkeypatch, name, rows):
    monkeypatch.setenv("FASSMVS_SWEEP_ROWS", rows)
    wl = scenegen.make_workload(name)
    p = wl["params"]
    level = p["n_levels"] - 1
    out = orc.run_frame(wl, keep=True, levels_only=level)
    lv = out["levels"][level]
    Ki, Kl, plan, H = _level_inputs(orc, wl, level)
    views = [hd.upload(pv[level]) for pv in out["pyr_views"]]
    ct = hd.stage_census(hd.upload(lv["img"]), p["census_w"], p["census_h"])
    assert np.array_equal(ct.numpy(), lv["ct"])
    got = hd.stage_cost(ct, views, wl["side"], p["census_w"], p["census_h"], plan["G"], plan["W"], H).numpy()
    assert_costs_from_images(got, lv["S"], f"{name} rows {rows}")


def test_cost_volume_with_windows(orc, hd):
    """Finer level of the small oblique scene with per-pixel windows taken
    from the oracle's own seed."""
    wl = scenegen.make_workload("config2_small")
    p = wl["params"]
    out = orc.run_frame(wl, keep=True, levels_only=1)
    lv = out["levels"][1]
    offs = out["levels"][2]["seed"]["offs"]
    Ki, Kl, plan, H = _level_inputs(orc, wl, 1)
    views = [hd.upload(pv[1]) for pv in out["pyr_views"]]
    ct = hd.upload(lv["ct"])
    got = hd.stage_cost(ct, views, wl["side"], p["census_w"], p["census_h"], plan["G"], plan["W"], H,
                        offs=hd.upload(offs)).numpy()
    assert_costs_from_images(got, lv["S"], "windows")


def _lut(orc, wl):
    p = wl["params"]
    m = orc.subset_multiplier(wl["side"])
    return m * p["p1"], orc.p2_lut(m * p["p1"], p["p2_mode"], m * p["p2_fixed"], p["p2_alpha"], p["p2_beta"])


@pytest.mark.parametrize("paths", [8, 4])
def test_sgm_top_level_bit_exact(orc, hd, paths):
    wl = scenegen.make_workload("config1")
    out = orc.run_frame(wl, keep=True)
    lv = out["levels"][0]
    p1, lut = _lut(orc, wl)
    S = lv["S"]
    Sbar, Lr = orc.sgm(S, [S.shape[2]], p1, lut, lv["img"], paths, want_lr=True)
    r = hd.stage_sgm(hd.upload(S), [S.shape[2]], p1, lut, hd.upload(lv["img"]), paths, want_lr=True,
                     want_sbar=True, want_wta=True)
    assert np.array_equal(r["Lr"].numpy(), Lr)
    assert np.array_equal(r["Sbar"].numpy(), Sbar)
    wta = r["wta"].numpy()
    assert np.array_equal(wta, np.argmin(Sbar, axis=-1))
    # fused path (no per-direction outputs kept) gives the same winner
    r2 = hd.stage_sgm(hd.upload(S), [S.shape[2]], p1, lut, hd.upload(lv["img"]), paths)
    assert np.array_equal(r2["wta"].numpy(), wta)
    assert np.array_equal(r2["c3"].numpy(), r["c3"].numpy())


def test_sgm_windows_sn_families_bit_exact(orc, hd):
    """Finer level with dynamic windows, surface-normal offsets and two
    plane families (config-3 shape), from the oracle's own inputs."""
    wl = scenegen.make_workload("config3_small")
    out = orc.run_frame(wl, keep=True, levels_only=1)
    lv = out["levels"][1]
    assert lv["offs"] is not None and lv["dI"] is not None
    p1, lut = _lut(orc, wl)
    W = lv["plan"]["W"]
    Sbar, Lr = orc.sgm(lv["S"], W, p1, lut, lv["img"], 8, offs=lv["offs"], dI=lv["dI"], want_lr=True)
    r = hd.stage_sgm(hd.upload(lv["S"]), W, p1, lut, hd.upload(lv["img"]), 8, offs=hd.upload(lv["offs"]),
                     dI=hd.upload(lv["dI"]), want_lr=True, want_sbar=True)
    assert np.array_equal(r["Lr"].numpy(), Lr)
    assert np.array_equal(r["Sbar"].numpy(), Sbar)
    assert np.array_equal(r["wta"].numpy(), np.argmin(Sbar, axis=-1))
    r2 = hd.stage_sgm(hd.upload(lv["S"]), W, p1, lut, hd.upload(lv["img"]), 8, offs=hd.upload(lv["offs"]),
                      dI=hd.upload(lv["dI"]))
    assert np.array_equal(r2["wta"].numpy(), r["wta"].numpy())


def test_refine_median_normals_conf(orc, hd):
    wl = scenegen.make_workload("config2_small")
    out = orc.run_frame(wl, keep=True, levels_only=1)
    lv = out["levels"][1]
    plan = lv["plan"]
    Ki, _ = orc.kinv_level(np.asarray(wl["K"]), 1)
    p1, lut = _lut(orc, wl)
    r = hd.stage_sgm(hd.upload(lv["S"]), plan["W"], p1, lut, hd.upload(lv["img"]), 8, offs=hd.upload(lv["offs"]),
                     dI=hd.upload(lv["dI"]))
    label, fam, depth = hd.stage_refine(r["wta"], r["c3"], plan["W"], plan["G"], plan["fam_n"],
                                        np.concatenate(plan["deltas"]), Ki, offs=hd.upload(lv["offs"]))
    assert np.array_equal(label.numpy(), lv["label"])
    assert np.array_equal(fam.numpy(), lv["fam"])
    d = depth.numpy()
    assert np.array_equal(d, lv["depth_raw"]) or np.max(np.abs(d - lv["depth_raw"]) / np.maximum(lv["depth_raw"], 1e-9)) < 1e-6
    med = hd.stage_median(hd.upload(lv["depth_raw"])).numpy()
    assert np.array_equal(med, lv["depth"])
    nraw, normal, conf = hd.stage_normals(hd.upload(lv["depth"]), hd.upload(lv["img"]), Ki, 2, 10.0,
                                          hd.upload(lv["label"]), hd.upload(lv["fam"]), plan["fam_n"], 60.0)
    # the smoothing weights come from a table the host evaluates with the
    # oracle's expression and libm, so the smoothed normals and the
    # confidence are the oracle's floats
    assert np.array_equal(nraw.numpy(), lv["normal_raw"]), first_mismatch(nraw.numpy(), lv["normal_raw"])
    assert np.array_equal(normal.numpy(), lv["normal"]), first_mismatch(normal.numpy(), lv["normal"])
    assert np.array_equal(conf.numpy(), lv["conf"]), first_mismatch(conf.numpy(), lv["conf"])


def test_seed_bit_exact(orc, hd):
    wl = scenegen.make_workload("config3_small")
    out = orc.run_frame(wl, keep=True, levels_only=1)
    coarse = out["levels"][2]
    seed = coarse["seed"]
    plan_f = orc.level_plan(wl, 1)
    Ki_f, _ = orc.kinv_level(np.asarray(wl["K"]), 1)
    fh, fw = out["levels"][1]["img"].shape
    dbar, nbar, offs, dI = hd.stage_seed(hd.upload(coarse["depth"]), hd.upload(coarse["normal"]), fw, fh, Ki_f,
                                         plan_f["fam_n"], plan_f["deltas"], plan_f["W"])
    assert np.array_equal(dbar.numpy(), seed["dbar"])
    assert np.array_equal(nbar.numpy(), seed["nbar"])
    assert np.array_equal(offs.numpy(), seed["offs"]), first_mismatch(offs.numpy(), seed["offs"])
    assert np.array_equal(dI.numpy(), seed["dI"]), first_mismatch(dI.numpy(), seed["dI"])


@pytest.mark.parametrize("name", ["config2_small_list", "config2_small_xr"])
def test_seed_bit_exact_on_lists_of_varying_spacing(orc, hd, name):
    """Windows and surface-normal offsets from plane lists that are not
    uniform in inverse distance (an explicit geometric list; the cross-ratio
    list): the continuous index is found by bisection on the GPU and by a
    scan in the oracle."""
    wl = scenegen.make_workload(name)
    out = orc.run_frame(wl, keep=True, levels_only=1)
    top = wl["params"]["n_levels"] - 1
    coarse = out["levels"][top]
    seed = coarse["seed"]
    plan_f = orc.level_plan(wl, top - 1)
    Ki_f, _ = orc.kinv_level(np.asarray(wl["K"]), top - 1)
    fh, fw = out["levels"][top - 1]["img"].shape
    inv = [1.0 / d for d in plan_f["deltas"]]
    assert any(np.ptp(np.diff(i)) > 1e-3 * abs(np.mean(np.diff(i))) for i in inv)   # really non-uniform
    dbar, nbar, offs, dI = hd.stage_seed(hd.upload(coarse["depth"]), hd.upload(coarse["normal"]), fw, fh, Ki_f,
                                         plan_f["fam_n"], plan_f["deltas"], plan_f["W"])
    assert np.array_equal(offs.numpy(), seed["offs"]), first_mismatch(offs.numpy(), seed["offs"])
    assert np.array_equal(dI.numpy(), seed["dI"]), first_mismatch(dI.numpy(), seed["dI"])
    assert np.count_nonzero(seed["dI"]) > 0


@pytest.mark.parametrize("kernel", ["packed", "one-label"])
@pytest.mark.parametrize("name,level", [("config2_small", 1), ("config3_small", 1), ("config1", 0)])
def test_sgm_path_gradient_bit_exact(orc, hd, monkeypatch, kernel, name, level):
    """SGM^Pi-pg: path costs and aggregate bit-exact with the oracle's
    path-gradient recursion (windows and plane families included), through
    the two-label and the one-label kernel."""
    monkeypatch.setenv("FASSMVS_SGM_UNPACKED", "1" if kernel == "one-label" else "0")
    wl = scenegen.make_workload(name)
    out = orc.run_frame(wl, keep=True, levels_only=level)
    lv = out["levels"][level]
    plan = lv["plan"]
    Ki, _ = orc.kinv_level(np.asarray(wl["K"]), level)
    p1, lut = _lut(orc, wl)
    fam_delta = np.concatenate(plan["deltas"])
    geom = dict(G=plan["G"], fam_delta=fam_delta, fam_n=plan["fam_n"], Kinv=Ki, step=plan["step"])
    Sbar, Lr = orc.sgm(lv["S"], plan["W"], p1, lut, lv["img"], 8, offs=lv["offs"], want_lr=True, pg=geom)
    r = hd.stage_sgm_pg(hd.upload(lv["S"]), plan["W"], plan["G"], p1, lut, hd.upload(lv["img"]), 8, fam_delta,
                        plan["fam_n"], Ki, plan["step"],
                        offs=hd.upload(lv["offs"]) if lv["offs"] is not None else None, want_lr=True,
                        want_sbar=True)
    assert np.array_equal(r["Lr"].numpy(), Lr)
    assert np.array_equal(r["Sbar"].numpy(), Sbar)
    assert np.array_equal(r["wta"].numpy(), np.argmin(Sbar, axis=-1))


@pytest.mark.parametrize("kernel", ["packed", "one-label"])
@pytest.mark.parametrize("shape,W,G,paths", [
    ((37, 53), [24, 16, 32], [40, 16, 64], 8),      # even windows, 72 labels
    ((37, 53), [23, 16, 9], [40, 16, 12], 8),       # odd windows (one-label kernel either way)
    ((21, 30), [200, 130], [260, 130], 8),          # 330 labels: three packed registers, ragged
    ((17, 23), [96, 96, 96, 96], [192, 96, 128, 160], 8),   # 384 labels in four families
    ((13, 19), [256, 200], [300, 200], 8),          # 456 labels: four packed registers
    ((19, 26), [128], [256], 4),                    # exactly 128 labels, four paths
    ((1, 41), [16, 8], [30, 8], 8),                 # one-row image
    ((33, 1), [16], [16], 8),                       # one-column image
])
def test_sgm_random_volumes(orc, hd, monkeypatch, kernel, shape, W, G, paths):
    """Random costs, window offsets over the whole plane list and
    surface-normal offsets over [-7, 7] (shifts reach far into and past the
    guards): path costs, aggregate and winners bit-exact with the oracle,
    for the packed two-label kernel and the one-label kernel."""
    if kernel == "one-label":
        monkeypatch.setenv("FASSMVS_SGM_UNPACKED", "1")
    else:
        monkeypatch.delenv("FASSMVS_SGM_UNPACKED", raising=False)
    h, w = shape
    rng = np.random.default_rng(sum(W) * 131 + h * 7 + w)
    F = len(W)
    D = int(sum(W))
    S = rng.integers(0, 64, (h, w, D), dtype=np.uint8)
    offs = np.stack([rng.integers(0, g - wf + 1, (h, w)) for g, wf in zip(G, W)]).astype(np.int32)
    dI = rng.integers(-7, 8, (8, h, w, F)).astype(np.int8)
    ref = rng.integers(0, 256, (h, w), dtype=np.uint8)
    p1 = 8
    lut = orc.p2_lut(p1, 1, 64, 8.0, 10.0)
    Sbar, Lr = orc.sgm(S, W, p1, lut, ref, paths, offs=offs, dI=dI, want_lr=True)
    r = hd.stage_sgm(hd.upload(S), W, p1, lut, hd.upload(ref), paths, offs=hd.upload(offs), dI=hd.upload(dI),
                     want_lr=True, want_sbar=True)
    assert np.array_equal(r["Lr"].numpy(), Lr)
    assert np.array_equal(r["Sbar"].numpy(), Sbar)
    assert np.array_equal(r["wta"].numpy(), np.argmin(Sbar, axis=-1))


@pytest.mark.parametrize("name", ["config1_ncc", "config2_small_ncc"])
def test_ncc_cost_from_oracle_warps_bit_exact(orc, hd, name):
    """NCC window sums, square root, scaling and the subset mean are
    bit-exact when the kernel is fed the oracle's warped images."""
    wl = scenegen.make_workload(name)
    p = wl["params"]
    level = p["n_levels"] - 1
    out = orc.run_frame(wl, keep=True, levels_only=level)
    lv = out["levels"][level]
    Ki, Kl, plan, H = _level_inputs(orc, wl, level)
    views = [pv[level] for pv in out["pyr_views"]]
    h, w = lv["img"].shape
    warped = np.zeros((len(views), sum(plan["G"]), h, w), np.float32)
    for k in range(len(views)):
        for g in range(sum(plan["G"])):
            warped[k, g] = orc.warp(views[k], H[k, g], w, h)
    got = hd.stage_cost_ncc(hd.upload(lv["img"]), None, wl["side"], p["census_w"], p["census_h"], plan["G"],
                            plan["W"], H, warped=hd.upload(warped)).numpy()
    assert np.array_equal(got, lv["S"])


@pytest.mark.parametrize("name", ["config1_ncc", "config2_small_ncc"])
@pytest.mark.parametrize("rows", ["4", "8"])
def test_ncc_cost_volume_from_images(orc, hd, monkeypatch, name, rows):
    monkeypatch.setenv("FASSMVS_SWEEP_ROWS", rows)
    wl = scenegen.make_workload(name)
    p = wl["params"]
    level = p["n_levels"] - 1
    out = orc.run_frame(wl, keep=True, levels_only=level)
    lv = out["levels"][level]
    Ki, Kl, plan, H = _level_inputs(orc, wl, level)
    views = [hd.upload(pv[level]) for pv in out["pyr_views"]]
    got = hd.stage_cost_ncc(hd.upload(lv["img"]), views, wl["side"], p["census_w"], p["census_h"], plan["G"],
                            plan["W"], H).numpy()
    assert_costs_from_images(got, lv["S"], f"{name} ncc rows {rows}")


@pytest.mark.parametrize("n", [3, 7, 9])
def test_ncc_window_sizes_bit_exact(orc, hd, n):
    """3x3, 7x7 and 9x9 NCC windows on random views and random homographies
    near the identity, with offsets (dynamic windows), from the oracle's
    warped images."""
    rng = np.random.default_rng(n)
    h, w = 45, 70
    ref = rng.integers(0, 256, (h, w)).astype(np.uint8)
    views = [rng.integers(0, 256, (h, w)).astype(np.uint8) for _ in range(3)]
    side = [-1, 1, 1]
    G, W = [12, 6], [5, 6]
    H = np.zeros((3, sum(G), 3, 3))
    for k in range(3):
        for g in range(sum(G)):
            H[k, g] = np.eye(3) + rng.normal(0, 0.002, (3, 3)) * np.array([[1, 1, 50], [1, 1, 50], [0.001, 0.001, 1]])
    offs = np.stack([rng.integers(0, g - wf + 1, (h, w)) for g, wf in zip(G, W)]).astype(np.int32)
    warped = np.zeros((3, sum(G), h, w), np.float32)
    for k in range(3):
        for g in range(sum(G)):
            warped[k, g] = orc.warp(views[k], H[k, g], w, h)
    exp = orc.ncc_cost_volume(ref, views, side, n, n, G, W, H, offs)
    got = hd.stage_cost_ncc(hd.upload(ref), None, side, n, n, G, W, H, offs=hd.upload(offs),
                            warped=hd.upload(warped)).numpy()
    assert np.array_equal(got, exp)
