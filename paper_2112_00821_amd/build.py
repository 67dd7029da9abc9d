"""Build libfassmvs.so (gfx950 HIP kernels + host runtime) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfassmvs.so")
SOURCES = ["k_image.hip", "k_sweep.hip", "k_sgm.hip", "k_post.hip", "runtime.hip", "server.hip"]
# sweep variants (window width, height, cost: 0 census, 1 NCC), one object
# each from k_sweep_inst.hip so they compile in parallel
SWEEP_VARIANTS = [(5, 5, 0), (9, 7, 0), (7, 7, 0), (3, 3, 0), (5, 5, 1), (9, 9, 1), (7, 7, 1), (3, 3, 1)]
# two-label SGM kernels by label pairs per lane, one object each from
# k_sgm_inst.hip
SGM_PAIRS = [1, 2, 3, 4]
ARCH = os.environ.get("FASSMVS_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # parity: no fused multiply-add where the reference semantics fix the
    # operation order (warp coordinates, refinement, seeds)
    "-ffp-contract=off",
    # never emit packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
]


def _units():
    units = [(src, os.path.splitext(src)[0], []) for src in SOURCES]
    for cw, ch, cost in SWEEP_VARIANTS:
        # census windows: without the IR load/store vectorizer the paired
        # LDS reads of a window row need fewer address adds (3 % fewer VALU
        # instructions in the census loop, the sweep about 0.5 % faster)
        extra = ["-mllvm", "-amdgpu-load-store-vectorizer=false"] if cost == 0 else []
        units.append(("k_sweep_inst.hip", f"k_sweep_{cw}x{ch}_{cost}",
                      [f"-DFMVS_CW={cw}", f"-DFMVS_CH={ch}", f"-DFMVS_COST={cost}", *extra]))
    for kp in SGM_PAIRS:
        units.append(("k_sgm_inst.hip", f"k_sgm_pk{kp}", [f"-DFMVS_KP={kp}"]))
    return units


def _compile(unit) -> str:
    src, name, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *CFLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    # heaviest first: the sweep variants and the SGM dominate the build
    order = sorted(units, key=lambda u: (u[0] not in ("k_sgm_inst.hip", "k_sweep_inst.hip", "k_sgm.hip"), u[1]))
    with ThreadPoolExecutor(max_workers=min(len(order), os.cpu_count() or 8)) as ex:
        objs = list(ex.map(_compile, order))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
