"""Uneven batch: sixteen frames of different resolution (640x480 ..
1920x1080), view count (2-5, unequal subsets included), plane count
(64-192, so one or two label pairs per lane) and pyramid depth (2 or 3).

Submitted as one batch on one handle (one sweep launch and one persistent
aggregation launch per level round, the whole batch replayed from a captured
graph), every frame's maps are identical to the same frame run alone, on
the graph's first capture, on its replay and without the graph; the same
holds with sixteen handles in flight together.  The coarsest level of four
frames (5 views in 3 + 2, 192 labels, 2 levels, 2 views) and every level of
two more match the oracle at the frame tests' gates."""
import copy
import os
import time

import numpy as np
import pytest

import scenegen
from parity_util import compare_level

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
def alone(fm, frames):
    """Each frame on a handle of its own (levels kept for the oracle test)."""
    out, handles = {}, {}
    for sd, wl in frames.items():
        h = fm.Handle(fm.config_from_params(wl["params"], keep_levels=1))
        out[sd] = h.run_frame(wl)
        handles[sd] = h
    yield out, handles
    for h in handles.values():
        h.close()


@pytest.fixture(scope="module")
def batched(fm, frames):
    """The sixteen frames as one batch: graph capture, replay, no graph."""
    wls = [frames[sd] for sd in scenegen.CONFIG4_SEEDS]
    res = {}
    with fm.Handle(fm.config_from_params(wls[0]["params"])) as h:
        t0 = time.perf_counter()
        res["first"] = h.run_batch(wls)        # tuning, capture, launch
        t1 = time.perf_counter()
        res["replay"] = h.run_batch(wls)
        t2 = time.perf_counter()
        res["tuning"] = h.batch_tuning()
        os.environ["FASSMVS_BATCH_GRAPH"] = "0"
        try:
            res["eager"] = h.run_batch(wls)
        finally:
            del os.environ["FASSMVS_BATCH_GRAPH"]
    # untuned, with one and with four frame groups
    for G, graph in ((1, "1"), (4, "1"), (4, "0")):
        os.environ.update(FASSMVS_BATCH_TUNE="0", FASSMVS_BATCH_GROUPS=str(G), FASSMVS_BATCH_GRAPH=graph)
        try:
            with fm.Handle(fm.config_from_params(wls[0]["params"])) as h:
                res[f"groups{G}_graph{graph}"] = h.run_batch(wls)
                # untuned: each frame level's own sweep tile height
                assert h.batch_tuning()["groups"] == G and h.batch_tuning()["rows_per_thread"] == 0
        finally:
            for k in ("FASSMVS_BATCH_TUNE", "FASSMVS_BATCH_GROUPS", "FASSMVS_BATCH_GRAPH"):
                del os.environ[k]
    print(f"batch of 16: first {1e3 * (t1 - t0):.1f} ms (tuning + capture), replay {1e3 * (t2 - t1):.1f} ms, "
          f"tuning {res['tuning']}")
    return res


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
def test_frame_same_alone_and_in_the_batch(alone, batched, sd):
    i = scenegen.CONFIG4_SEEDS.index(sd)
    for run in ("first", "replay", "eager", "groups1_graph1", "groups4_graph1", "groups4_graph0"):
        for k in ("depth", "normal", "conf"):
            assert np.array_equal(alone[0][sd][k], batched[run][i][k]), (sd, run, k)
    assert np.mean(alone[0][sd]["depth"] > 0) > 0.5


def test_batch_tuning_reported(batched):
    t = batched["tuning"]
    assert t["rows_per_thread"] in (0, 4, 8) and t["sweep_blocks"] in (8192, 16384) and t["groups"] in (1, 2, 4, 8, 16)
    assert t["batch_ms"] > 0


def test_frames_in_flight_on_sixteen_handles(fm, frames, alone):
    handles = {sd: fm.Handle(fm.config_from_params(wl["params"])) for sd, wl in frames.items()}
    try:
        tickets = {sd: handles[sd].submit_frame(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"])
                   for sd, wl in frames.items()}
        for sd, wl in frames.items():
            d, n, c = _maps(wl)
            handles[sd].poll(tickets[sd], d, n, c)
            assert np.array_equal(d, alone[0][sd]["depth"]) and np.array_equal(n, alone[0][sd]["normal"])
            assert np.array_equal(c, alone[0][sd]["conf"])
    finally:
        for h in handles.values():
            h.close()


@pytest.mark.parametrize("sd", ORACLE_SEEDS)
def test_batch_coarsest_level_matches_oracle(orc, frames, alone, sd):
    wl = frames[sd]
    top = wl["params"]["n_levels"] - 1
    ref = orc.run_frame(wl, keep=True, levels_only=top)["levels"][top]
    h = alone[1][sd]
    lab = h.level_map(top, 4)
    dep = h.level_map(top, 0)
    agree = lab == ref["label"]
    assert agree.mean() >= 0.999, agree.mean()
    ok = agree & (ref["depth"] > 0)
    rel = np.abs(dep[ok] - ref["depth"][ok]) / ref["depth"][ok]
    assert np.mean(rel <= 1e-3) >= 0.999, np.max(rel)


def test_batch_of_mixed_small_frames_and_fallback_aggregation(fm):
    """Frames of one batch whose aggregation cannot share the persistent
    launch (path-gradient SGM) run it frame by frame; a shape change
    recaptures; each frame equals its run alone."""
    for variant in (1, 2):
        wls = []
        for name in ("config2_small", "config2_ragged", "config3_small"):
            wl = copy.deepcopy(scenegen.make_workload(name))
            wl["params"]["sgm_variant"] = variant
            wls.append(wl)
        ones = []
        for wl in wls:
            with fm.Handle(fm.config_from_params(wl["params"])) as h1:
                ones.append(h1.run_frame(wl))
        with fm.Handle(fm.config_from_params(wls[0]["params"])) as h:
            for order in ([0, 1, 2], [2, 1], [0, 1, 2]):
                got = h.run_batch([wls[i] for i in order])
                for i, g in zip(order, got):
                    for k in ("depth", "normal", "conf"):
                        assert np.array_equal(g[k], ones[i][k]), (variant, wls[i]["name"], k)


def test_batch_of_frames_with_many_labels(fm):
    """Frames whose levels take three and four packed label registers (four
    families of 96 and of 120 labels) in the batch's persistent aggregation:
    each frame equals its run alone."""
    wls = []
    for name, count in (("config3_small", 96), ("config3_small", 120)):
        wl = copy.deepcopy(scenegen.make_workload(name))
        for f in wl["families"]:
            f["count"] = count
        wl["params"]["window_labels"] = count
        wls.append(wl)
    ones = []
    for wl in wls:
        with fm.Handle(fm.config_from_params(wl["params"])) as h1:
            ones.append(h1.run_frame(wl))
    with fm.Handle(fm.config_from_params(wls[0]["params"])) as h:
        got = h.run_batch(wls)
    for i, g in enumerate(got):
        for k in ("depth", "normal", "conf"):
            assert np.array_equal(g[k], ones[i][k]), (wls[i]["name"], k)
        assert np.mean(ones[i]["depth"] > 0) > 0.5


def test_batch_replay_with_new_images(fm, monkeypatch):
    """A batch replayed from its captured group graphs (untuned: graphs on,
    two frame groups) reads the images of the current submission: the same
    shapes with other images give the maps of those images run alone."""
    monkeypatch.setenv("FASSMVS_BATCH_TUNE", "0")
    monkeypatch.setenv("FASSMVS_BATCH_GROUPS", "2")
    monkeypatch.delenv("FASSMVS_BATCH_GRAPH", raising=False)
    base = [scenegen.make_workload(n) for n in ("config2_small", "config2_ragged", "config3_small")]

    def variant(wl, k):
        w2 = copy.deepcopy(wl)
        for im in [w2["ref"]] + w2["views"]:
            im["img"] = np.ascontiguousarray(np.roll(im["img"], 3 * k, axis=1))
        return w2

    sets = [[variant(wl, k) for wl in base] for k in range(3)]
    with fm.Handle(fm.config_from_params(base[0]["params"])) as h:
        got = [h.run_batch(ws) for ws in sets]
        t = h.batch_tuning()
        assert t["graph"] and t["groups"] == 2
    for k, ws in enumerate(sets):
        for i, wl in enumerate(ws):
            with fm.Handle(fm.config_from_params(wl["params"])) as h1:
                one = h1.run_frame(wl)
            for key in ("depth", "normal", "conf"):
                assert np.array_equal(got[k][i][key], one[key]), (k, wl["name"], key)
    assert not np.array_equal(got[0][0]["depth"], got[1][0]["depth"])


def test_batch_errors(fm, frames):
    wl = frames[scenegen.CONFIG4_SEEDS[0]]
    with fm.Handle(fm.config_from_params(wl["params"])) as h:
        with pytest.raises(fm.FassmvsError) as e:
            h.submit_batch([])
        assert e.value.status == fm.EINVAL
        t = h.submit_batch([wl])
        with pytest.raises(fm.FassmvsError) as e:
            h.submit_frame(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"])
        assert e.value.status == fm.EBUSY
        with pytest.raises(fm.FassmvsError) as e:
            h.submit_batch([wl])
        assert e.value.status == fm.EBUSY
        d, n, c = _maps(wl)
        with pytest.raises(fm.FassmvsError) as e:
            h.poll_batch(t, 1, d)
        assert e.value.status == fm.EINVAL
        with pytest.raises(fm.FassmvsError) as e:
            h.poll_batch(t + 5, 0, d)
        assert e.value.status == fm.ENOTFOUND
        assert h.poll_batch(t, 0, d, n, c) == fm.OK
        ref = h.run_frame(wl)                              # the handle is free again
        assert np.array_equal(ref["depth"], d)
        bad = dict(wl, params=dict(wl["params"], n_levels=9))
        with pytest.raises(fm.FassmvsError) as e:
            h.submit_batch([wl, bad])
        assert e.value.status == fm.EINVAL


def test_batch_with_device_inputs_and_outputs(fm, frames, alone):
    """Device-resident images in and device maps out give the host path's
    maps."""
    sds = scenegen.CONFIG4_SEEDS[:5]
    wls = [frames[sd] for sd in sds]
    with fm.Handle(fm.config_from_params(wls[0]["params"])) as h:
        dev = [dict(wl, ref=dict(wl["ref"], img=h.upload(wl["ref"]["img"])),
                    views=[dict(v, img=h.upload(v["img"])) for v in wl["views"]]) for wl in wls]
        t = h.submit_batch(dev, mem_kind=fm.MEM_DEVICE)
        for i, (sd, wl) in enumerate(zip(sds, wls)):
            d = h.empty((wl["height"], wl["width"]), np.float32)
            c = h.empty((wl["height"], wl["width"]), np.float32)
            h.poll_batch(t, i, d, None, c, mem_kind=fm.MEM_DEVICE)
            assert np.array_equal(d.numpy(), alone[0][sd]["depth"]) and np.array_equal(c.numpy(), alone[0][sd]["conf"])


def test_batch_of_the_most_frames(fm):
    """64 frames (the most a batch takes) of 20 different widths: each equals
    its run alone; 65 frames are refused."""
    wl = scenegen.make_workload("config1")

    def crop(w):
        return dict(wl, width=w, ref=dict(wl["ref"], img=np.ascontiguousarray(wl["ref"]["img"][:, :w])),
                    views=[dict(v, img=np.ascontiguousarray(v["img"][:, :w])) for v in wl["views"]])

    shapes = [crop(160 - 4 * (i % 20)) for i in range(64)]
    with fm.Handle(fm.config_from_params(wl["params"])) as h:
        alone = {}
        for x in shapes[:20]:
            alone[x["width"]] = h.run_frame(x)
        got = h.run_batch(shapes)
        for x, g in zip(shapes, got):
            for k in ("depth", "normal", "conf"):
                assert np.array_equal(g[k], alone[x["width"]][k]), (x["width"], k)
        with pytest.raises(fm.FassmvsError) as e:
            h.submit_batch(shapes + shapes[:1])
        assert e.value.status == fm.EINVAL


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sd", [112, 107])
def test_batch_frame_every_level_matches_oracle(frames, alone, oracle_run, sd):
    """Every level of two config4 frames (640x480: 2 views, 168 labels, 3
    levels; 4 views, 184 labels, 2 levels) against the oracle's whole-frame
    run (started in a process of its own when the session starts); the
    batch gives these frames' maps bit for bit (above)."""
    wl = frames[sd]
    z = oracle_run(f"config4_{sd}")
    h = alone[1][sd]
    n = wl["params"]["n_levels"]
    for l in range(n - 1, -1, -1):
        got = dict(label=h.level_map(l, 4), depth=h.level_map(l, 0), normal=h.level_map(l, 2), conf=h.level_map(l, 3))
        exp = dict(label=z[f"l{l}_label"], depth=z[f"l{l}_depth"], normal=z[f"l{l}_normal"], conf=z[f"l{l}_conf"])
        rep = compare_level(got, exp, wl["params"]["normal_radius"])
        print(f"[batch] config4_{sd} level {l}: {rep}", flush=True)
        if l < n - 1:
            nf = len(wl["families"])
            assert np.mean(h.level_map(l, 6, n_fam=nf) == z[f"l{l}_offs"]) >= 0.999
            assert np.mean(h.level_map(l, 7, n_fam=nf) == z[f"l{l}_dI"]) >= 0.999
