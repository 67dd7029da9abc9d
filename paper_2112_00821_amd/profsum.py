"""Summarise rocprofv3 CSV output of bench.py runs into a short text profile.

Inputs are the directories rocprofv3 wrote with ``--output-format csv -o run``:
a ``--kernel-trace --stats`` run, a ``--pmc FETCH_SIZE`` run, a ``--pmc
WRITE_SIZE`` run and a ``--pmc`` run of SQ/GRBM counters.  The byte counters
are calibrated by the library's plain copy kernel (k_copy16, which reads and
writes every byte once) from the same runs: the factor is the copy's known
bytes over what the counter reads for it.

Usage::

    python3 -m paper_2112_00821_amd.profsum --trace T --fetch F --write W --sq S \
        --bench B.json --kernel k_sweep --workload "..." --command "..." --out profiles/x.md
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# sources each timed kernel is built from, and the build script that holds
# its compiler flags (the hash marks the counters stale once any of them
# changes)
KERNEL_SOURCES = {
    "k_sweep": ["csrc/k_sweep.hpp", "csrc/k_sweep.hip", "csrc/k_sweep_inst.hip", "csrc/dev_common.hpp",
                "csrc/kernels.hpp", "build.py"],
    "k_sgm": ["csrc/k_sgm.hpp", "csrc/k_sgm.hip", "csrc/dev_common.hpp", "csrc/kernels.hpp", "build.py"],
    "k_sgm_pk": ["csrc/k_sgm.hpp", "csrc/k_sgm_inst.hip", "csrc/dev_common.hpp", "csrc/kernels.hpp", "build.py"],
    "k_wta16": ["csrc/k_sgm.hpp", "csrc/k_sgm.hip", "csrc/dev_common.hpp", "csrc/kernels.hpp", "build.py"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("fmvs::", "")
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0]


def _base(name: str) -> str:
    return short_name(name).split("<")[0]


def read_stats(d):
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_stats.csv"))))
    return [(short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e6, float(r["TotalDurationNs"]) / 1e6,
             float(r["Percentage"])) for r in rows]


def read_counters(d):
    """Per dispatch: {dispatch_id: (kernel short name, grid, {counter: value})}."""
    out = {}
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        did = int(r["Dispatch_Id"])
        ent = out.setdefault(did, [short_name(r["Kernel_Name"]), int(r["Grid_Size"]), collections.Counter()])
        ent[2][r["Counter_Name"]] += float(r["Counter_Value"])
    return out


def per_kernel_avg(disp, counter):
    acc = collections.defaultdict(list)
    for name, _, c in disp.values():
        if counter in c:
            acc[name].append(c[counter])
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def calibration(disp, counter, copy_bytes):
    """Known bytes / counter bytes of the largest k_copy16 dispatch."""
    best = None
    for name, grid, c in disp.values():
        if name.startswith("k_copy16") and counter in c:
            if best is None or c[counter] > best:
                best = c[counter]
    if best is None or best <= 0:
        return None, None
    return copy_bytes / (best * 1024.0), best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--bench")
    ap.add_argument("--kernel", action="append", default=[],
                    help="kernel(s) whose traffic record the summary carries (default k_sweep)")
    ap.add_argument("--copy-mb", type=int, default=256)
    ap.add_argument("--workload", default="")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    kernels = a.kernel or ["k_sweep"]
    stats = read_stats(a.trace)
    lines = [f"# {', '.join(kernels)}: {a.workload}", "", "Commands (run from the repository root):", ""]
    lines += [f"    {c}" for c in a.command]
    lines += ["", "## Kernel time (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg ms | total ms | % |", "|---|---|---|---|---|"]
    for n, calls, avg, tot, pct in stats:
        lines.append(f"| {n} | {calls} | {avg:.4f} | {tot:.3f} | {pct:.2f} |")

    copy_bytes = a.copy_mb << 20
    traffic = {}
    if a.fetch and a.write:
        fd, wd = read_counters(a.fetch), read_counters(a.write)
        ff, fcal_raw = calibration(fd, "FETCH_SIZE", copy_bytes)
        wf, wcal_raw = calibration(wd, "WRITE_SIZE", copy_bytes)
        favg, fn = per_kernel_avg(fd, "FETCH_SIZE")
        wavg, wn = per_kernel_avg(wd, "WRITE_SIZE")
        avg_ms = {}
        for n, calls, avg, tot, pct in stats:
            avg_ms[n] = avg
        lines += ["", "## HBM bytes per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
                  f"Calibration: k_copy16 of {a.copy_mb} MiB reads FETCH_SIZE {fcal_raw:.0f} KiB and WRITE_SIZE "
                  f"{wcal_raw:.0f} KiB; factors {ff:.4f} (fetch) and {wf:.4f} (write) scale the counters to bytes.",
                  "", "| kernel | dispatches | fetch MB | write MB | total MB | avg ms | GB/s |",
                  "|---|---|---|---|---|---|---|"]
        for k in sorted(favg, key=lambda k: -(favg[k] + wavg.get(k, 0.0))):
            if k.startswith("k_copy16") or k.startswith("__amd"):
                continue
            fb = favg[k] * 1024.0 * ff
            wb = wavg.get(k, 0.0) * 1024.0 * wf
            ms = avg_ms.get(k)
            gbs = (fb + wb) / (ms / 1e3) / 1e9 if ms else float("nan")
            lines.append(f"| {k} | {fn[k]} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} | "
                         f"{ms if ms else float('nan'):.4f} | {gbs:.0f} |")
            traffic[k] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb, "fetch_n": fn[k],
                          "write_n": wn.get(k, 0)}
        # the summarised kernels by grid size (one row per distinct launch
        # shape, e.g. per pyramid level)
        by_grid = collections.defaultdict(lambda: [0.0, 0.0, 0])
        for d, (name, grid, c) in fd.items():
            if _base(name) in kernels and "FETCH_SIZE" in c:
                by_grid[(name, grid)][0] += c["FETCH_SIZE"] * 1024.0 * ff
                by_grid[(name, grid)][2] += 1
        for d, (name, grid, c) in wd.items():
            if _base(name) in kernels and "WRITE_SIZE" in c and (name, grid) in by_grid:
                by_grid[(name, grid)][1] += c["WRITE_SIZE"] * 1024.0 * wf
        if by_grid:
            lines += ["", "By launch shape (grid size in work-items; the same shape is the same pyramid level):", "",
                      "| kernel | grid | dispatches | fetch MB | write MB | total MB |", "|---|---|---|---|---|---|"]
            for (name, grid), (fb, wb, n) in sorted(by_grid.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
                lines.append(f"| {name} | {grid} | {n} | {fb / n / 1e6:.1f} | {wb / n / 1e6:.1f} | "
                             f"{(fb + wb) / n / 1e6:.1f} |")

    if a.sq:
        sd = read_counters(a.sq)
        names = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU",
                 "SQ_INSTS_VMEM_RD", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"]
        avgs = {n: per_kernel_avg(sd, n)[0] for n in names}
        lines += ["", "## Instruction counters per dispatch (rocprofv3 --pmc SQ_* GRBM_GUI_ACTIVE)", "",
                  "GRBM_GUI_ACTIVE is summed over the 8 XCDs.  VALU busy = SQ_INSTS_VALU / (32 x GRBM_GUI_ACTIVE): "
                  "an XCD's 128 SIMDs retire at most 32 wave64 VALU instructions per cycle.  The clock is "
                  "GRBM_GUI_ACTIVE / 8 over the traced average duration.", "",
                  "| kernel | VALU instr | LDS instr | VMEM rd | VALU busy | clock GHz |", "|---|---|---|---|---|---|"]
        avg_ms = {n: avg for n, calls, avg, tot, pct in stats}
        for k in sorted(avgs["SQ_INSTS_VALU"], key=lambda k: -avgs["SQ_INSTS_VALU"][k]):
            v = avgs["SQ_INSTS_VALU"][k]
            g = avgs["GRBM_GUI_ACTIVE"].get(k, 0.0)
            busy = v / (32.0 * g) if g else float("nan")
            ms = avg_ms.get(k)
            clk = g / 8.0 / (ms / 1e3) / 1e9 if (ms and g) else float("nan")
            lines.append(f"| {k} | {v:.3e} | {avgs['SQ_INSTS_LDS'].get(k, 0):.3e} | "
                         f"{avgs['SQ_INSTS_VMEM_RD'].get(k, 0):.3e} | {busy:.3f} | {clk:.2f} |")

    if a.bench:
        txt = open(a.bench).read().strip().splitlines()
        js = json.loads([l for l in txt if l.startswith("{")][-1])
        lines += ["", "## Bench line of the same build", "", "    " + json.dumps(js)]

    recs = []
    for kern in kernels:
        # per launch over every instantiation of the kernel (the frame's
        # launches may use several, e.g. one tile height per level), as the
        # benchmark averages its launch times; the instantiation with the
        # most traffic is named
        inst = sorted((k for k in traffic if _base(k) == kern), key=lambda k: -traffic[k]["bytes"])
        nf = sum(traffic[k]["fetch_n"] for k in inst)
        nw = sum(traffic[k]["write_n"] for k in inst)
        if inst and nf and nw:
            fetch = sum(traffic[k]["fetch_bytes"] * traffic[k]["fetch_n"] for k in inst) / nf
            write = sum(traffic[k]["write_bytes"] * traffic[k]["write_n"] for k in inst) / nw
            recs.append({"kernel": kern, "instantiation": inst[0], "instantiations": inst,
                         "source_hash": source_hash(kern), "traffic_bytes_per_launch": fetch + write,
                         "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write})
    if recs:
        lines += ["", "## Traffic records read by bench.py", ""]
        lines += ["traffic_json: " + json.dumps(r) for r in recs]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_traffic(path: str, kernel: str):
    """Traffic per launch from a committed profile, or None when missing or
    when the kernel's sources changed since the counters were taken."""
    try:
        for line in open(path):
            if line.startswith("traffic_json: "):
                rec = json.loads(line[len("traffic_json: "):])
                if rec.get("kernel") == kernel and rec.get("source_hash") == source_hash(kernel):
                    return rec
    except OSError:
        return None
    return None


if __name__ == "__main__":
    main()
