"""Run the oracle on one named workload in a process of its own and save its
per-level maps as an .npz (test infrastructure: the full-size parity tests
start these jobs when the test session starts, so the oracle's minutes of
single-threaded work overlap the GPU tests).

    python tests/oracle_frame_job.py <workload> <out.npz> [levels_only]
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KEYS = ("label", "fam", "depth", "depth_raw", "normal", "conf")


def main(name, out_path, levels_only=None):
    import oracle
    import scenegen
    oracle.build()
    wl = scenegen.make_workload(name)
    out = oracle.run_frame(wl, keep=True, levels_only=levels_only)
    arrs = {}
    for l, lv in out["levels"].items():
        for k in KEYS:
            arrs[f"l{l}_{k}"] = lv[k]
        for k in ("offs", "dI"):
            if lv.get(k) is not None:
                arrs[f"l{l}_{k}"] = lv[k]
        if "seed" in lv:
            for k in ("offs", "dI"):
                if lv["seed"].get(k) is not None:
                    arrs[f"l{l}_seed_{k}"] = lv["seed"][k]
        if l == 0:
            arrs["l0_S"] = lv["S"]
    tmp = out_path + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, out_path)


if __name__ == "__main__":
    lv = int(sys.argv[3]) if len(sys.argv) > 3 else None
    main(sys.argv[1], sys.argv[2], lv)
