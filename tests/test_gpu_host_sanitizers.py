"""The library's host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer: `fassmvs_host_check` (built by
paper_2112_00821_amd/build_host_check.py with both sanitizers on the host
code of runtime.hip and server.hip; device code is not instrumented) drives frames with host and device
buffers, explicit plane lists and depth ranges, a batch of uneven frames,
the served form with two streams, the plane-set helpers and error paths on
device 0.  Any sanitizer report aborts it."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2112_00821_amd", "fassmvs_host_check")


def test_host_runtime_under_asan_and_ubsan():
    assert os.path.exists(EXE), "fassmvs_host_check is not built (paper_2112_00821_amd/build_host_check.py builds it)"
    # No quarantine of freed chunks (freed memory stays poisoned until it is
    # reused): with one, a thread's quarantine cache is handed back when the
    # thread exits, and a runtime thread exiting after the HIP runtime has
    # unloaded then returns device allocations to it -- an AddressSanitizer
    # CHECK at teardown, not a report on this code.
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:quarantine_size_mb=0:thread_local_quarantine_size_kb=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "host check: ok" in r.stdout, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
