"""Served form: a frame's maps are the same alone and in the mix of several
streams running concurrently, and the same as the plain pipeline's on the
same bundle; keyframe selection, admission and error paths."""
import numpy as np
import pytest

import scenegen
from parity_util import compare_level

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    import paper_2112_00821_amd as fm
    return fm


@pytest.fixture(scope="module")
def streams():
    return [scenegen.served_stream(seed, w, h, 5, spacing=0.6, planes=32)
            for seed, w, h in [(210, 320, 184), (211, 400, 240), (212, 256, 160)]]


def _cfg(fm, st):
    return fm.config_from_params(st["params"])


def _run(fm, streams, order, n_slots, cfg):
    """Submit frames in the given order [(stream index, frame index)];
    returns {(stream, frame): (result, maps)}."""
    out = {}
    with fm.Server(cfg, n_slots=n_slots) as srv:
        sid = {i: srv.open_stream(st["K"], st["width"], st["height"], st["families"]) for i, st in enumerate(streams)}
        rid = {}
        for s, f in order:
            img, R, t = streams[s]["frames"][f]
            rid[srv.submit(sid[s], img, R, t)] = (s, f)
        for _ in range(len(order)):
            r = srv.next(-1)
            s, f = rid[r["request_id"]]
            maps = srv.fetch(r["request_id"], r["width"], r["height"]) if r["status"] == fm.OK else None
            out[(s, f)] = (r, maps)
    return out


def test_same_alone_and_in_the_mix(fm, streams):
    cfg = _cfg(fm, streams[0])
    alone = _run(fm, streams[:1], [(0, f) for f in range(5)], 1, cfg)
    order = []
    for f in range(5):
        for s in (1, 0, 2):
            order.append((s, f))
    mix = _run(fm, streams, order, 3, cfg)
    n_ok = 0
    for f in range(5):
        ra, ma = alone[(0, f)]
        rm, mm = mix[(0, f)]
        assert ra["status"] == rm["status"]
        assert ra["n_views"] == rm["n_views"] and ra["keyframe"] == rm["keyframe"]
        if ma is not None:
            n_ok += 1
            for k in ("depth", "normal", "conf"):
                assert np.array_equal(ma[k], mm[k]), (f, k)
    assert n_ok == 4
    # keyframe rule restated: a frame is a keyframe when its camera centre is
    # at least 1 m from the last keyframe's; it is matched against the
    # keyframes before it (at most 4)
    keys, exp_key, exp_views = [], [], []
    for f in range(5):
        _, R, t = streams[0]["frames"][f]
        C = -R.T @ t
        exp_views.append(min(len(keys), 4))
        k = not keys or np.linalg.norm(C - keys[-1]) >= 1.0
        exp_key.append(int(k))
        if k:
            keys.append(C)
    assert [alone[(0, f)][0]["keyframe"] for f in range(5)] == exp_key
    assert [alone[(0, f)][0]["n_views"] for f in range(5)] == exp_views
    assert alone[(0, 0)][0]["status"] == fm.ENOTFOUND


def test_served_frame_equals_plain_pipeline(fm, orc, streams):
    """A served frame's maps equal the plain pipeline's on the same bundle
    (the frame and the keyframes it was matched against), and that bundle's
    maps match the oracle's at every level."""
    st = streams[0]
    cfg = _cfg(fm, st)
    served = _run(fm, [st], [(0, f) for f in range(4)], 2, cfg)
    # frame 3 was matched against the keyframes before it, most recent first
    keys = []
    for f in range(3):
        _, R, t = st["frames"][f]
        C = -R.T @ t
        if not keys or np.linalg.norm(C - keys[-1][1]) >= 1.0:
            keys.append((f, C))
    kf = [f for f, _ in keys][::-1]
    assert served[(0, 3)][0]["n_views"] == len(kf)
    img, R, t = st["frames"][3]
    ref = dict(img=img, R=R, t=t)
    views = [dict(img=st["frames"][k][0], R=st["frames"][k][1], t=st["frames"][k][2]) for k in kf]
    wl = dict(K=st["K"], width=st["width"], height=st["height"], ref=ref, views=views, side=[-1] * len(kf),
              families=st["families"], params=st["params"])
    oref = orc.run_frame(wl, keep=True)
    with fm.Handle(fm.config_from_params(st["params"], keep_levels=1)) as h:
        tk = h.submit_frame(ref, views, [-1] * len(kf), st["K"], st["families"])
        d = np.zeros((st["height"], st["width"]), np.float32)
        n = np.zeros((st["height"], st["width"], 3), np.float32)
        c = np.zeros((st["height"], st["width"]), np.float32)
        h.poll(tk, d, n, c)
        for l in range(st["params"]["n_levels"]):
            got = dict(label=h.level_map(l, 4), depth=h.level_map(l, 0), normal=h.level_map(l, 2),
                       conf=h.level_map(l, 3))
            compare_level(got, oref["levels"][l], st["params"]["normal_radius"])
    maps = served[(0, 3)][1]
    assert np.array_equal(maps["depth"], d)
    assert np.array_equal(maps["normal"], n)
    assert np.array_equal(maps["conf"], c)


def test_footprint_admission_serialises_under_a_tight_budget(fm, streams):
    """A budget that holds one frame's footprint only: frames still all
    complete (one at a time), with the same maps."""
    st = streams[0]
    cfg = _cfg(fm, st)
    import ctypes as C
    fams = (fm.PlaneFamily * 1)()
    f0 = st["families"][0]
    fams[0].n[:] = list(f0["n"])
    fams[0].delta_min, fams[0].delta_max, fams[0].count = f0["delta_min"], f0["delta_max"], f0["count"]
    fp = C.c_uint64()
    assert fm.lib().fassmvs_frame_footprint(C.byref(cfg), st["width"], st["height"], 4, fams, 1,
                                            C.byref(fp)) == fm.OK
    ref = _run(fm, [st], [(0, f) for f in range(5)], 3, cfg)
    with fm.Server(cfg, n_slots=3, hbm_budget_bytes=fp.value + 1) as srv:
        sid = srv.open_stream(st["K"], st["width"], st["height"], st["families"])
        ids = [srv.submit(sid, *st["frames"][f]) for f in range(5)]
        got = {}
        for _ in range(5):
            r = srv.next(-1)
            if r["status"] == fm.OK:
                got[ids.index(r["request_id"])] = srv.fetch(r["request_id"], r["width"], r["height"])
    assert sorted(got) == [1, 2, 3, 4]
    for f in got:
        assert np.array_equal(got[f]["depth"], ref[(0, f)][1]["depth"])


def test_admission_counts_held_memory_with_mixed_frame_sizes(fm, streams):
    """Two stream sizes on three slots under a budget just above one large
    frame's footprint: admission counts what the slots' pipelines hold (a
    slot that ran a large frame keeps its buffers) plus the growth a frame
    needs, so no frame fails for memory, and the maps are those of a run
    without a budget."""
    import ctypes as C
    big, small = streams[1], streams[2]
    cfg = _cfg(fm, big)
    fams = fm._families(big["families"])
    fp = C.c_uint64()
    assert fm.lib().fassmvs_frame_footprint(C.byref(cfg), big["width"], big["height"], 4, fams, 1,
                                            C.byref(fp)) == fm.OK
    order = []
    for f in range(5):
        order += [(0, f), (1, f)]
    pair = [big, small]
    ref = _run(fm, pair, order, 3, cfg)
    out = {}
    with fm.Server(cfg, n_slots=3, hbm_budget_bytes=fp.value + 1) as srv:
        sid = {i: srv.open_stream(st["K"], st["width"], st["height"], st["families"]) for i, st in enumerate(pair)}
        rid = {}
        for s, f in order:
            rid[srv.submit(sid[s], *pair[s]["frames"][f])] = (s, f)
        for _ in range(len(order)):
            r = srv.next(-1)
            out[rid[r["request_id"]]] = (r, srv.fetch(r["request_id"], r["width"], r["height"])
                                         if r["status"] == fm.OK else None)
    for key, (r, maps) in out.items():
        r0, m0 = ref[key]
        assert r["status"] == r0["status"], (key, r["status"])
        assert r["status"] in (fm.OK, fm.ENOTFOUND)
        if maps is not None:
            for k in ("depth", "normal", "conf"):
                assert np.array_equal(maps[k], m0[k]), (key, k)
    assert sum(r["status"] == fm.OK for r, _ in out.values()) == 8


def test_server_errors(fm, streams):
    st = streams[0]
    cfg = _cfg(fm, st)
    with fm.Server(cfg, n_slots=1) as srv:
        with pytest.raises(fm.FassmvsError) as e:
            srv.submit(99, *st["frames"][0])
        assert e.value.status == fm.ENOTFOUND
        sid = srv.open_stream(st["K"], st["width"], st["height"], st["families"])
        srv.close_stream(sid)
        with pytest.raises(fm.FassmvsError):
            srv.submit(sid, *st["frames"][0])
        assert srv.next(0) is None
    with pytest.raises(fm.FassmvsError):
        fm.Server(cfg, n_slots=0)
