"""Build fassmvs_host_check: the library's host runtime (runtime.hip,
server.hip) rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer on
its host code only (device code is never instrumented), linked with the
kernel objects of the library build and a driver (csrc/host_check.cpp) into
one executable.  Run after build.py (it reuses that build's objects)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import build as lib_build  # noqa: E402

HOST_CHECK = os.path.join(lib_build.PKG, "fassmvs_host_check")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(lib_build.BUILD, "san"), exist_ok=True)
    host = {"runtime.hip": "runtime_san", "server.hip": "server_san", "host_check.cpp": "host_check"}
    units = [(src, os.path.join("san", name), SAN) for src, name in host.items()]
    with ThreadPoolExecutor(max_workers=len(units)) as ex:
        san_objs = list(ex.map(lib_build._compile, units))
    kernels = [os.path.join(lib_build.BUILD, name + ".o") for _, name, _ in lib_build._units()
               if name not in ("runtime", "server")]
    missing = [o for o in kernels if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"kernel objects missing (run build.py first): {missing[:3]}")
    tmp = HOST_CHECK + ".tmp"
    cmd = [lib_build.HIPCC, f"--offload-arch={lib_build.ARCH}", *SAN, "-o", tmp, *san_objs, *kernels,
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host check link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, HOST_CHECK)
    if verbose:
        print("built", HOST_CHECK)
    return HOST_CHECK


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
