import os
import subprocess
import sys
import tempfile
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# oracle runs the parity tests compare with: workload -> (last level run or
# None for the whole frame, the test file that needs it), each in a process
# of its own, started as soon as the session knows that file is selected
ORACLE_JOBS = {"config2": (None, "test_gpu_fullsize"), "config3": (2, "test_gpu_fullsize"),
               "config4_112": (None, "test_gpu_batch"), "config4_107": (None, "test_gpu_batch")}
_jobs = {}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def pytest_collection_finish(session):
    files = {f for _, f in ORACLE_JOBS.values() if any(f in item.nodeid for item in session.items)}
    if not files:
        return
    import oracle
    oracle.build()
    tmp = tempfile.mkdtemp(prefix="fassmvs_oracle_")
    for name, (lv, f) in ORACLE_JOBS.items():
        if f not in files:
            continue
        out = os.path.join(tmp, f"{name}.npz")
        cmd = [sys.executable, os.path.join(ROOT, "tests", "oracle_frame_job.py"), name, out]
        if lv is not None:
            cmd.append(str(lv))
        log = open(os.path.join(tmp, f"{name}.log"), "w")
        _jobs[name] = (subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), out, log, time.time())


def pytest_sessionfinish(session, exitstatus):
    for proc, _, log, _ in _jobs.values():
        if proc.poll() is None:
            proc.kill()
            proc.wait()
        log.close()


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def oracle_run():
    """oracle_run(name) -> the oracle's per-level maps of that workload
    (np.load of the job's .npz), waiting for its job to finish."""
    import numpy as np

    def get(name, timeout=900):
        proc, out, log, t0 = _jobs[name]
        print(f"[oracle job] waiting for {name}", flush=True)
        while True:
            try:
                rc = proc.wait(timeout=20)
                break
            except subprocess.TimeoutExpired:
                el = time.time() - t0
                print(f"[oracle job] {name} still running after {el:.0f} s", flush=True)
                if el > timeout:
                    proc.kill()
                    raise
        log.flush()
        if rc != 0:
            with open(log.name) as f:
                raise RuntimeError(f"oracle job {name} failed ({rc}):\n{f.read()[-3000:]}")
        print(f"[oracle job] {name} done after {time.time() - t0:.0f} s", flush=True)
        return np.load(out, allow_pickle=False)

    return get
