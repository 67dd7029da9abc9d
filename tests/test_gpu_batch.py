"""Uneven batch: sixteen frames of different resolution (640x480 ..
1920x1080), view count (2-5, unequal subsets included), plane count
(64-192, so one or two label pairs per lane) and pyramid depth (2 or 3)
in flight on the device together, one pipeline handle (own stream) each.

Every frame's maps are identical to the same frame run alone; the coarsest
level of four of them (5 views in 3 + 2, 192 labels, 2 levels, 2 views)
matches the oracle at the frame tests' gates."""
import time

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu

ORACLE_SEEDS = [104, 105, 107, 112]


@pytest.fixture(scope="module")
def fm():
    import paper_2112_00821_amd as fm
    return fm


@pytest.fixture(scope="module")
def frames():
    return {sd: scenegen.make_workload(f"config4_{sd}") for sd in scenegen.CONFIG4_SEEDS}


def _maps(wl):
    h, w = wl["height"], wl["width"]
    return (np.zeros((h, w), np.float32), np.zeros((h, w, 3), np.float32), np.zeros((h, w), np.float32))


@pytest.fixture(scope="module")
def runs(fm, frames):
    """(alone, together, handles kept for level maps) for every frame."""
    alone = {}
    t0 = time.perf_counter()
    for sd, wl in frames.items():
        with fm.Handle(fm.config_from_params(wl["params"])) as h:
            alone[sd] = h.run_frame(wl)
    t_alone = time.perf_counter() - t0
    handles = {sd: fm.Handle(fm.config_from_params(wl["params"], keep_levels=1)) for sd, wl in frames.items()}
    t0 = time.perf_counter()
    tickets = {sd: handles[sd].submit_frame(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"])
               for sd, wl in frames.items()}
    together = {}
    for sd, wl in frames.items():
        d, n, c = _maps(wl)
        handles[sd].poll(tickets[sd], d, n, c)
        together[sd] = dict(depth=d, normal=n, conf=c)
    t_together = time.perf_counter() - t0
    print(f"16 uneven frames: one at a time {t_alone * 1e3:.1f} ms (first use of each handle included), "
          f"all in flight {t_together * 1e3:.1f} ms")
    yield alone, together, handles
    for h in handles.values():
        h.close()


def test_shapes_are_uneven(frames):
    sizes = {(wl["width"], wl["height"]) for wl in frames.values()}
    views = {len(wl["views"]) for wl in frames.values()}
    planes = {wl["families"][0]["count"] for wl in frames.values()}
    levels = {wl["params"]["n_levels"] for wl in frames.values()}
    assert len(sizes) == 4 and views == {2, 3, 4, 5} and levels == {2, 3}
    assert min(planes) <= 128 < max(planes)
    for wl in frames.values():
        nl = sum(1 for s in wl["side"] if s < 0)
        assert nl - (len(wl["side"]) - nl) in (0, 1)   # split as evenly as possible, the extra one on the left


@pytest.mark.parametrize("sd", scenegen.CONFIG4_SEEDS)
def test_frame_same_alone_and_in_the_batch(runs, sd):
    alone, together, _ = runs
    for k in ("depth", "normal", "conf"):
        assert np.array_equal(alone[sd][k], together[sd][k]), (sd, k)
    assert np.mean(alone[sd]["depth"] > 0) > 0.5


@pytest.mark.parametrize("sd", ORACLE_SEEDS)
def test_batch_coarsest_level_matches_oracle(orc, frames, runs, sd):
    wl = frames[sd]
    top = wl["params"]["n_levels"] - 1
    ref = orc.run_frame(wl, keep=True, levels_only=top)["levels"][top]
    h = runs[2][sd]
    lab = h.level_map(top, 4)
    dep = h.level_map(top, 0)
    agree = lab == ref["label"]
    assert agree.mean() >= 0.999, agree.mean()
    ok = agree & (ref["depth"] > 0)
    rel = np.abs(dep[ok] - ref["depth"][ok]) / ref["depth"][ok]
    assert np.mean(rel <= 1e-3) >= 0.999, np.max(rel)
