#!/usr/bin/env python3
"""Throughput benchmark of the FaSS-MVS hot path on one MI355X.

One step = one whole coarse-to-fine frame (pyramid, reference census, fused
warp+census+Hamming sweep, 8-path surface-aware SGM with fused WTA,
refinement, median, normals, confidence, coarse-to-fine seeding) of the
1920x1080 oblique UAV-shaped workload (reference + 4 views, 3 levels x 128
planes, census 9x7), with the input images already resident in HBM.  Prints
one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpx·hyp/s (sweep+SGM), frames/s, p50/p99 latency: served vs plain, 1 MI355X"
PEAK_HBM_GBS = 8000.0
# plain 32-bit VALU lane operations: 256 CUs x 64 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic work of the sweep per (pixel, hypothesis, view): one compare per
# census bit of the warped window, XOR + popcount of the 62-bit words (3), and
# the warp of one sample (projective map + bilinear, about 15 operations)
SWEEP_ALG_OPS_9x7 = 62 + 3 + 15
# NCC 5x5: per window sample a sum, a square and a product (3), about 20 for
# the correlation coefficient and its scaling, the warp of one sample (15)
SWEEP_ALG_OPS_NCC5 = 3 * 25 + 20 + 15
# algorithmic bytes of SGM per (pixel, hypothesis): S read once per path (8 x
# 1 B) plus the aggregate written and read once (2 x 2 B)
SGM_ALG_BYTES = 12.0
# bytes of this design per (pixel, hypothesis): S read by each of the 8
# direction walks (8 x 1 B), each direction's uint16 path costs written once
# and read once by the streaming winner-takes-all (2 x 8 x 2 B)
SGM_DESIGN_BYTES = 40.0
PROFILE = os.path.join(ROOT, "profiles", "k_sweep_config2.md")
SGM_PROFILE = os.path.join(ROOT, "profiles", "k_sgm_pk_config2.md")

WORKLOADS = {
    "config2": ("1920x1080 oblique urban scene, reference + 4 views (2 left, 2 right), 3 levels x 128 "
                "fronto-parallel planes over [20, 400] m (window 128 below the top), census 9x7, "
                "SGM^Pi-sn 8 paths, adaptive P2, parabola refinement, 5x5 median, normals, confidence"),
    "config1": "160x120 reference + 2 views, 32 planes, census 5x5, 8-path SGM P1=8 P2=64, 1 level",
    "config2_ncc": ("the 1920x1080 workload above matched with the negated, truncated, scaled NCC 5x5 "
                    "(phi1 = 100, adaptive P2)"),
    "config2_pg": "the 1920x1080 workload above with SGM^Pi-pg (path-gradient index jump) at every level",
    "config3": ("2704x1520 reference + 4 views of the same scene generator, 4 plane families (fronto, ground "
                "normal, ground normal tilted +-20 deg) x 96 planes per level, 3 levels, census 9x7, SGM^Pi-sn"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--host-io-steps", type=int, default=5,
                    help="after the timed region, run this many frames with host input/output buffers and report "
                         "that PCIe-inclusive rate beside the device-resident one")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served-vs-plain measurement on the four-stream trace")
    ap.add_argument("--served-slots", type=int, default=2)
    ap.add_argument("--served-frames", type=int, default=130,
                    help="distinct rendered frames per stream (13 s of each stream's flight at 10 Hz)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes rendering the synthetic inputs")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the sixteen uneven config4 frames (one batch, one at a time, all in flight)")
    ap.add_argument("--batch-repeats", type=int, default=3)
    ap.add_argument("--no-config3", action="store_true", help="skip the 2704x1520 four-family frame section")
    ap.add_argument("--config3-steps", type=int, default=5)
    ap.add_argument("--timeline", default="", help="write the last timed frame's stage timeline (JSON) here")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before timing, copy this many MiB device-to-device once (a plain copy kernel of known "
                         "size whose HBM byte counters calibrate the profiler's FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the hot path does not shard across GPUs); got --gpus {args.gpus}",
              file=sys.stderr)
        return 2

    import scenegen

    # every synthetic input is rendered on the CPU, in worker processes
    # forked before the GPU is touched
    names = [args.workload]
    if not args.no_config3 and args.workload != "config3":
        names.append("config3")
    if not args.no_batch:
        names += [f"config4_{sd}" for sd in scenegen.CONFIG4_SEEDS]
    wls, served_streams = render_inputs(scenegen, names, 0 if args.no_served else args.served_frames, args.workers)

    import paper_2112_00821_amd as fm

    wl = wls[args.workload]
    m = measure(fm, wl, args.steps, args.warmup, args.host_io_steps, args.calib_copy_mb)
    h, w = wl["height"], wl["width"]
    ms = m["ms"]
    hyp = m["work"]["pixel_hyp"]
    times, times0 = m["times"], m["times0"]
    value = hyp / 1e6 / (ms / 1e3)
    sweep_ms = times["sweep"][0] / max(times["sweep"][1], 1)
    sweep_launches = times["sweep"][1] / args.steps
    sgm_ms = (times["sgm_dirs"][0] + times["sgm_wta"][0]) / args.steps
    sweep_frame_ms = times["sweep"][0] / args.steps
    ks_value = hyp / 1e6 / ((sweep_frame_ms + sgm_ms) / 1e3)
    # dominant kernel and its roofline
    from paper_2112_00821_amd import profsum
    if sweep_frame_ms >= sgm_ms:
        units = m["work"]["pixel_hyp_views"] / sweep_launches
        alg_ops = SWEEP_ALG_OPS_NCC5 if wl["params"].get("cost") == "ncc" else SWEEP_ALG_OPS_9x7
        achieved = alg_ops * units / (sweep_ms / 1e3) / 1e12
        tr = profsum.read_traffic(PROFILE, "k_sweep") if args.workload == "config2" else None
        roof = {"bound": "alu", "kernel": "k_sweep", "achieved": achieved, "peak": PEAK_VALU_TOPS,
                "unit": "TOP/s", "frac": achieved / PEAK_VALU_TOPS,
                "traffic": tr["traffic_bytes_per_launch"] if tr else None,
                "avg_launch_ms": sweep_ms, "launches_per_frame": sweep_launches,
                "alg_ops_per_px_hyp_view": alg_ops}
    else:
        achieved = SGM_ALG_BYTES * hyp / (sgm_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_sgm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None, "stage_ms_per_frame": sgm_ms,
                "alg_bytes_per_px_hyp": SGM_ALG_BYTES}
    sgm_roof = sgm_roofline(m, args.steps)
    # counted HBM bytes per launch of the aggregation and WTA kernels, from
    # the committed profile while their sources are unchanged
    if args.workload == "config2":
        for kern in ("k_sgm_pk", "k_wta16"):
            tr = profsum.read_traffic(SGM_PROFILE, kern)
            sgm_roof[f"traffic_{kern}"] = tr["traffic_bytes_per_launch"] if tr else None
    lat_ms = np.array(m["lat"]) * 1e3
    host_ms = m["host_ms"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpx·hyp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ("f64 NCC window sums, u8/u16 costs, f32 warp, f64 geometry" if wl["params"].get("cost") == "ncc"
                  else "u8/u16 integer matching, f32 warp, f64 geometry"), "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "pixel_hyp_per_frame": hyp,
                   "width": w, "height": h},
        "frames_per_s": round(1e3 / ms, 2),
        "ms_per_step_profiled": round(m["profiled_ms"], 3),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3), "mode": "plain per-frame pipeline"},
        "sweep_sgm_only_value": round(ks_value, 1),
        "host_io": ({"ms_per_frame": round(host_ms, 3), "value": round(hyp / 1e6 / (host_ms / 1e3), 1),
                     "unit": "Mpx·hyp/s", "note": "host buffers in and out (PCIe included); not the headline value"}
                    if host_ms else None),
        "stage_ms_per_frame": {k: round(v[0] / args.steps, 4) for k, v in times.items() if v[1]},
        "stage_ms_per_frame_level0": {k: round(v[0] / args.steps, 4) for k, v in times0.items() if v[1]},
        "sweep_label_inflation": round(m["work"]["sweep_evaluated"] / hyp, 4) if hyp else None,
        "roofline": roof,
        "sgm_roofline": sgm_roof,
    }
    if args.timeline:
        with open(args.timeline, "w") as f:
            json.dump({"workload": args.workload, "steps": [
                {"stage": st, "level": lv, "start_ms": round(a, 4), "ms": round(d, 4)}
                for st, lv, a, d in m["timeline"]]}, f, indent=1)
    if "config3" in wls and args.workload != "config3":
        out["config3"] = frame_section(fm, wls["config3"], args.config3_steps)
    if served_streams is not None:
        out["served"] = served_bench(fm, served_streams, args.served_slots)
    if not args.no_batch:
        out["batch"] = batch_bench(fm, [wls[f"config4_{sd}"] for sd in scenegen.CONFIG4_SEEDS], args.batch_repeats)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))
    return 0


def measure(fm, wl, steps, warmup, host_io_steps=0, calib_copy_mb=0):
    """Time `steps` frames of a workload on one handle (inputs and outputs
    in HBM, the frame replayed from its captured graph) after `warmup`
    untimed ones; then the same frames on a profiling handle for the
    per-stage and per-level device times (HIP-event timers, which keep the
    frame out of a graph)."""
    h, w = wl["height"], wl["width"]
    res = {}
    for profile in (0, 1):
        cfg = fm.config_from_params(wl["params"], profile=profile)
        with fm.Handle(cfg) as hd:
            ref = dict(wl["ref"], img=hd.upload(wl["ref"]["img"]))
            views = [dict(v, img=hd.upload(v["img"])) for v in wl["views"]]
            depth = hd.empty((h, w), np.float32)
            normal = hd.empty((h, w, 3), np.float32)
            conf = hd.empty((h, w), np.float32)

            if calib_copy_mb and profile == 0:
                nb = calib_copy_mb << 20
                a_ = hd.empty((nb,), np.uint8).fill(1)
                b_ = hd.empty((nb,), np.uint8)
                fm.lib().fassmvs_memcpy(hd.h, b_.vp, a_.vp, nb, 2)
                del a_, b_

            def step():
                t = hd.submit_frame(ref, views, wl["side"], wl["K"], wl["families"], mem_kind=fm.MEM_DEVICE)
                hd.poll(t, depth, normal, conf, mem_kind=fm.MEM_DEVICE, wait_ms=-1)

            for _ in range(warmup if profile == 0 else 1):
                step()
            hd.synchronize()
            hd.reset_stage_times()
            lat = []
            t0 = time.perf_counter()
            for _ in range(steps):
                a = time.perf_counter()
                step()
                lat.append(time.perf_counter() - a)
            hd.synchronize()
            el = time.perf_counter() - t0
            if profile == 0:
                res.update(ms=el / steps * 1e3, lat=lat, host_ms=None)
                # the same frames handed over as host buffers (PCIe upload of
                # the images and download of the three output maps included)
                if host_io_steps:
                    dh = np.zeros((h, w), np.float32)
                    nh = np.zeros((h, w, 3), np.float32)
                    ch = np.zeros((h, w), np.float32)
                    hd.synchronize()
                    t1 = time.perf_counter()
                    for _ in range(host_io_steps):
                        t = hd.submit_frame(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"])
                        hd.poll(t, dh, nh, ch, wait_ms=-1)
                    res["host_ms"] = (time.perf_counter() - t1) / host_io_steps * 1e3
            else:
                res.update(profiled_ms=el / steps * 1e3, times=hd.stage_times(), times0=hd.stage_times_level(0),
                           work=hd.frame_work(), timeline=hd.frame_timeline())
    return res


def sgm_roofline(m, steps):
    """The aggregation's bandwidth over all levels and at full resolution
    only, by the method's bytes and by this design's."""
    hyp = m["work"]["pixel_hyp"]
    times, times0 = m["times"], m["times0"]
    sgm_ms = (times["sgm_dirs"][0] + times["sgm_wta"][0]) / steps
    r = {"bound": "hbm", "stages": "sgm_dirs + sgm_wta", "ms_per_frame": sgm_ms, "peak": PEAK_HBM_GBS,
         "unit": "GB/s", "alg_bytes_per_px_hyp": SGM_ALG_BYTES,
         "achieved_alg": SGM_ALG_BYTES * hyp / (sgm_ms / 1e3) / 1e9,
         "design_bytes_per_px_hyp": SGM_DESIGN_BYTES,
         "achieved_design": SGM_DESIGN_BYTES * hyp / (sgm_ms / 1e3) / 1e9}
    r["frac_alg"] = r["achieved_alg"] / PEAK_HBM_GBS
    r["frac_design"] = r["achieved_design"] / PEAK_HBM_GBS
    # full resolution only (the coarser levels' volumes partly stay in cache)
    hyp0 = m["work"]["pixel_hyp_level"][0]
    sgm0_ms = (times0["sgm_dirs"][0] + times0["sgm_wta"][0]) / steps
    if sgm0_ms > 0:
        r["level0"] = {
            "ms_per_frame": round(sgm0_ms, 4), "sgm_dirs_ms": round(times0["sgm_dirs"][0] / steps, 4),
            "sgm_wta_ms": round(times0["sgm_wta"][0] / steps, 4), "pixel_hyp": hyp0,
            "achieved_alg": SGM_ALG_BYTES * hyp0 / (sgm0_ms / 1e3) / 1e9,
            "frac_alg": SGM_ALG_BYTES * hyp0 / (sgm0_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
            "design_bytes_per_px_hyp": SGM_DESIGN_BYTES,
            "frac_design": SGM_DESIGN_BYTES * hyp0 / (sgm0_ms / 1e3) / 1e9 / PEAK_HBM_GBS}
    return r


def frame_section(fm, wl, steps):
    """A secondary workload's figures: frame time, throughput, stages and
    the aggregation's bandwidth (1 warm-up frame, `steps` timed)."""
    m = measure(fm, wl, steps, 1)
    hyp = m["work"]["pixel_hyp"]
    return {"workload": f"{wl['name']}: {WORKLOADS.get(wl['name'], '')}", "steps": steps,
            "ms_per_frame": round(m["ms"], 3), "frames_per_s": round(1e3 / m["ms"], 2),
            "value": round(hyp / 1e6 / (m["ms"] / 1e3), 1), "unit": "Mpx·hyp/s", "pixel_hyp_per_frame": hyp,
            "stage_ms_per_frame": {k: round(v[0] / steps, 4) for k, v in m["times"].items() if v[1]},
            "stage_ms_per_frame_level0": {k: round(v[0] / steps, 4) for k, v in m["times0"].items() if v[1]},
            "sgm_roofline": sgm_roofline(m, steps)}


def _render_workload(name):
    import scenegen
    wl = scenegen.make_workload(name)
    wl.pop("scene", None)
    wl.pop("gt", None)
    return name, wl


_SERVED_PATHS = None


def _render_one(job):
    import scenegen
    s, i = job
    return s, i, scenegen.served_image(_SERVED_PATHS[s], i)


def render_inputs(scenegen, names, served_frames, workers):
    """The named workloads and the four served streams (config-5 sizes,
    served_frames distinct frames each along the stream's flight path),
    rendered by `workers` processes (forked before the GPU is touched),
    largest jobs first."""
    import multiprocessing as mp
    global _SERVED_PATHS
    _SERVED_PATHS = ([scenegen.served_path(seed, w, h, served_frames) for seed, w, h in scenegen.SERVED_STREAMS]
                     if served_frames else [])
    jobs = [("wl", n) for n in names] + [("img", (s, i)) for s in reversed(range(len(_SERVED_PATHS)))
                                           for i in range(served_frames)]
    wls, imgs = {}, {}

    def take(kind, res):
        if kind == "wl":
            wls[res[0]] = res[1]
        else:
            imgs[(res[0], res[1])] = res[2]

    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            pending = [(kind, pool.apply_async(_render_workload if kind == "wl" else _render_one, (arg,)))
                       for kind, arg in jobs]
            for kind, r in pending:
                take(kind, r.get())
    else:
        for kind, arg in jobs:
            take(kind, _render_workload(arg) if kind == "wl" else _render_one(arg))
    streams = None
    if served_frames:
        streams = []
        for s, p in enumerate(_SERVED_PATHS):
            frames = [(imgs[(s, i)], p["poses"][i][0], p["poses"][i][1]) for i in range(served_frames)]
            streams.append(dict(K=p["K"], width=p["width"], height=p["height"], families=p["families"],
                                params=p["params"], frames=frames))
    return wls, streams


def _trace(streams, rate_hz=10.0, seed=300, first=None):
    """Arrivals of every stream's frames (the first `first` of each, or all)
    at rate_hz with exponential jitter (mean 5 ms)."""
    rng = np.random.default_rng(seed)
    ev = []
    for s, st in enumerate(streams):
        F = len(st["frames"]) if first is None else min(first, len(st["frames"]))
        last = -1.0
        for i in range(F):
            t = i / rate_hz + rng.exponential(0.005)
            t = max(t, last + 1e-3)
            last = t
            ev.append((t, s, i))
    ev.sort()
    return ev


def _run_trace(fm, srv, streams, events, speed):
    """Submit the trace to the server at its arrival times divided by speed
    (speed 0: all at once).  Returns throughput and latency figures."""
    import threading
    sids = {}
    expected = len(events)
    done = []

    def collect():
        while len(done) < expected:
            r = srv.next(-1)
            r["t_done"] = time.perf_counter()
            if r["status"] == fm.OK:
                srv.fetch(r["request_id"], r["width"], r["height"])
            done.append(r)

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    for (t, s, i) in events:
        if s not in sids:
            st = streams[s]
            sids[s] = srv.open_stream(st["K"], st["width"], st["height"], st["families"])
        if speed > 0:
            dt = t0 + t / speed - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        srv.submit(sids[s], *streams[s]["frames"][i])
    th.join()
    for sid in sids.values():
        srv.close_stream(sid)
    t_end = max(r["t_done"] for r in done)
    ok = [r for r in done if r["status"] == fm.OK]
    lat = np.array([r["latency_ms"] for r in ok])
    span = t_end - t0
    hyp = 0.0
    for r in ok:
        w, h = r["width"], r["height"]
        hyp += sum((w >> l) * (h >> l) * 128 for l in range(3))
    return {"frames": len(ok), "seconds": round(span, 3), "frames_per_s": round(len(ok) / span, 2),
            "mpx_hyp_per_s": round(hyp / 1e6 / span, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                           "p99": round(float(np.percentile(lat, 99)), 2),
                           "max": round(float(lat.max()), 2)}}


def served_bench(fm, streams, n_slots):
    """Served vs plain on the config-5 trace: the same server with one slot
    (the plain sequential per-frame pipeline) and with n_slots concurrent
    slots.  After an untimed pass over each stream's first frames that sizes
    every buffer pool, the whole trace runs at its real arrival rate (10 Hz
    per stream) and all at once (sustained rate)."""
    cfg = fm.config_from_params(streams[0]["params"])
    events = _trace(streams)
    warm = _trace(streams, first=6)
    F = len(streams[0]["frames"])
    out = {"streams": [f"{st['width']}x{st['height']}" for st in streams],
           "trace": f"{len(events)} distinct rendered frames: 4 streams x {F} frames ({F / 10:.1f} s of each "
                    f"stream's flight) at 10 Hz (+exp. jitter, mean 5 ms), keyframe every 1 m at 0.5 m spacing, "
                    f"up to 4 keyframes per bundle, 3 levels x 128 planes, census 9x7, SGM^Pi-sn",
           "slots": n_slots}
    for name, k in (("plain", 1), ("served", n_slots)):
        with fm.Server(cfg, n_slots=k) as srv:
            _run_trace(fm, srv, streams, warm, 0)        # warm-up: allocations
            out[name] = {"realtime": _run_trace(fm, srv, streams, events, 1.0),
                         "saturated": _run_trace(fm, srv, streams, events, 0)}
    return out


def batch_bench(fm, frames, repeats):
    """The sixteen uneven frames (config4 shapes), inputs in HBM, one handle
    each (buffers allocated by an untimed first pass): one frame at a time
    (submit, wait, next) against all sixteen submitted at once and then
    collected.  Best of `repeats` passes each."""
    hyp = 0.0
    for wl in frames:
        D, L = wl["families"][0]["count"], wl["params"]["n_levels"]
        hyp += sum((wl["width"] >> l) * (wl["height"] >> l) * D for l in range(L))
    handles = [fm.Handle(fm.config_from_params(wl["params"])) for wl in frames]
    try:
        inputs = []
        for h, wl in zip(handles, frames):
            ref = dict(wl["ref"], img=h.upload(wl["ref"]["img"]))
            views = [dict(v, img=h.upload(v["img"])) for v in wl["views"]]
            hh, ww = wl["height"], wl["width"]
            outs = (h.empty((hh, ww), np.float32), h.empty((hh, ww, 3), np.float32), h.empty((hh, ww), np.float32))
            inputs.append((ref, views, outs))

        def submit(i):
            ref, views, _ = inputs[i]
            wl = frames[i]
            return handles[i].submit_frame(ref, views, wl["side"], wl["K"], wl["families"], mem_kind=fm.MEM_DEVICE)

        def wait(i, t):
            d, n, c = inputs[i][2]
            handles[i].poll(t, d, n, c, mem_kind=fm.MEM_DEVICE)

        for i in range(len(frames)):   # allocations
            wait(i, submit(i))
        best_seq = best_all = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            for i in range(len(frames)):
                wait(i, submit(i))
            best_seq = min(best_seq, time.perf_counter() - t0)
            t0 = time.perf_counter()
            tickets = [submit(i) for i in range(len(frames))]
            for i, t in enumerate(tickets):
                wait(i, t)
            best_all = min(best_all, time.perf_counter() - t0)
        # one batch on one handle: per level round one sweep launch and one
        # persistent aggregation launch for all frames, replayed as a graph
        bh = fm.Handle(fm.config_from_params(frames[0]["params"]))
        try:
            wls = [dict(wl, ref=inputs[i][0], views=inputs[i][1]) for i, wl in enumerate(frames)]

            def run_batch():
                t = bh.submit_batch(wls, mem_kind=fm.MEM_DEVICE)
                for i in range(len(frames)):
                    d, n, c = inputs[i][2]
                    bh.poll_batch(t, i, d, n, c, mem_kind=fm.MEM_DEVICE)

            run_batch()   # tuning, capture
            tuning = bh.batch_tuning()
            best_batch = float("inf")
            for _ in range(repeats):
                t0 = time.perf_counter()
                run_batch()
                best_batch = min(best_batch, time.perf_counter() - t0)
            os.environ["FASSMVS_BATCH_GRAPH"] = "0"
            best_eager = float("inf")
            try:
                for _ in range(repeats):
                    t0 = time.perf_counter()
                    run_batch()
                    best_eager = min(best_eager, time.perf_counter() - t0)
            finally:
                del os.environ["FASSMVS_BATCH_GRAPH"]
        finally:
            bh.close()
    finally:
        for h in handles:
            h.close()
    res = {"frames": len(frames), "pixel_hyp": hyp, "batch_tuning": tuning}
    for name, t in (("one_at_a_time", best_seq), ("all_in_flight", best_all), ("one_batch_graph", best_batch),
                    ("one_batch_eager", best_eager)):
        res[name] = {"ms": round(t * 1e3, 2), "frames_per_s": round(len(frames) / t, 1),
                     "mpx_hyp_per_s": round(hyp / 1e6 / t, 1)}
    return res


def cpu_baseline(wl, min_seconds=10.0, max_runs=5):
    """The oracle, single-threaded, on a bounded sample of the same frame:
    its coarsest pyramid level (every stage of that level), repeated until
    about ten seconds of CPU work are timed."""
    import oracle
    oracle.build()
    top = wl["params"]["n_levels"] - 1
    runs = 0
    t0 = time.perf_counter()
    while True:
        out = oracle.run_frame(wl, keep=False, levels_only=top)
        runs += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or runs >= max_runs:
            break
    lv = out["levels"][top]
    hh, ww = lv["depth"].shape
    plan = oracle.level_plan(wl, top)
    hyp = hh * ww * sum(plan["W"]) * runs
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(hyp / 1e6 / el, 3), "unit": "Mpx·hyp/s", "cores": 1, "kind": "oracle",
            "host_cpu": cpu, "host_threads_visible": os.cpu_count(),
            "sample": f"coarsest level of the same frame ({ww}x{hh} x {sum(plan['W'])} planes, pyramid + "
                      f"census + cost volume + 8-path SGM + refinement + median + normals + confidence), "
                      f"{runs} run(s), {el:.1f} s single-threaded"}


if __name__ == "__main__":
    sys.exit(main())
