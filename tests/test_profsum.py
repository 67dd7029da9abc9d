"""The profile summariser: counter scaling by the copy kernel, the traffic
records bench.py reads back, and that the committed records match the
current kernel sources (so the benchmark line carries counted traffic)."""
import csv
import os
import subprocess
import sys

import pytest

from paper_2112_00821_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_sources_exist():
    for kern, files in profsum.KERNEL_SOURCES.items():
        for rel in files:
            assert os.path.isfile(os.path.join(os.path.dirname(profsum.__file__), rel)), (kern, rel)


@pytest.mark.parametrize("profile,kernel", [
    ("k_sweep_config2.md", "k_sweep"),
    ("k_sgm_pk_config2.md", "k_sgm_pk"),
    ("k_sgm_pk_config2.md", "k_wta16"),
])
def test_committed_records_match_sources(profile, kernel):
    rec = profsum.read_traffic(os.path.join(ROOT, "profiles", profile), kernel)
    if rec is None:
        # the benchmark then reports traffic null; the profile's recorded
        # commands regenerate it on the GPU
        pytest.skip(f"{profile}: the traffic record of {kernel} predates the current kernel sources")
    assert rec["traffic_bytes_per_launch"] == pytest.approx(
        rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, counter, copy_kib, kern_kib):
    os.makedirs(d)
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    rows = [[1, "void fmvs::k_copy16(uint4 const*, uint4*, unsigned long)", 1024, counter, copy_kib]]
    # two dispatches of the measured kernel, counters split over two rows each
    for did, kib in ((2, kern_kib), (3, kern_kib * 3)):
        rows.append([did, "void fmvs::k_sweep<9, 7, 8, false, 0>(fmvs::SweepArgs)", 4096, counter, kib / 2])
        rows.append([did, "void fmvs::k_sweep<9, 7, 8, false, 0>(fmvs::SweepArgs)", 4096, counter, kib / 2])
    _write(os.path.join(d, "run_counter_collection.csv"), hdr, rows)


def test_counters_scaled_by_the_copy_kernel(tmp_path):
    mb = 4
    copy_bytes = mb << 20
    # the copy reads copy_bytes but FETCH_SIZE shows half of it; WRITE_SIZE all
    _counters(tmp_path / "fetch", "FETCH_SIZE", copy_bytes / 2 / 1024, 1000.0)
    _counters(tmp_path / "write", "WRITE_SIZE", copy_bytes / 1024, 500.0)
    os.makedirs(tmp_path / "trace")
    _write(tmp_path / "trace" / "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"],
           [["void fmvs::k_sweep<9, 7, 8, false, 0>(fmvs::SweepArgs)", 2, 2.0e6, 4.0e6, 100.0]])
    out = tmp_path / "p.md"
    subprocess.run([sys.executable, "-m", "paper_2112_00821_amd.profsum", "--trace", str(tmp_path / "trace"),
                    "--fetch", str(tmp_path / "fetch"), "--write", str(tmp_path / "write"), "--copy-mb", str(mb),
                    "--kernel", "k_sweep", "--workload", "synthetic", "--out", str(out)], check=True, cwd=ROOT)
    rec = profsum.read_traffic(str(out), "k_sweep")
    # per dispatch on average: fetch (1000 + 3000) / 2 KiB x 2, write (500 + 1500) / 2 KiB x 1
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(1000 * 1024 * 1.0)
    assert rec["instantiation"] == "k_sweep<9, 7, 8, false, 0>"
    txt = out.read_text()
    assert "factors 2.0000 (fetch) and 1.0000 (write)" in txt


def test_traffic_record_averages_over_instantiations(tmp_path):
    """A frame's launches of one kernel may use several instantiations (a
    tile height per level): the record is per launch over all of them."""
    mb = 4
    copy_bytes = mb << 20
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    k8 = "void fmvs::k_sweep<9, 7, 8, false, 0>(fmvs::SweepArgs)"
    k4 = "void fmvs::k_sweep<9, 7, 4, false, 0>(fmvs::SweepArgs)"
    for counter, copy_kib, vals in (("FETCH_SIZE", copy_bytes / 2 / 1024, (600.0, 300.0, 30.0)),
                                    ("WRITE_SIZE", copy_bytes / 1024, (900.0, 450.0, 60.0))):
        d = tmp_path / counter
        os.makedirs(d)
        rows = [[1, "void fmvs::k_copy16(uint4 const*, uint4*, unsigned long)", 1024, counter, copy_kib],
                [2, k8, 4096, counter, vals[0]], [3, k8, 2048, counter, vals[1]], [4, k4, 1024, counter, vals[2]]]
        _write(os.path.join(d, "run_counter_collection.csv"), hdr, rows)
    os.makedirs(tmp_path / "trace")
    _write(tmp_path / "trace" / "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"],
           [[k8, 2, 2.0e6, 4.0e6, 90.0], [k4, 1, 0.4e6, 0.4e6, 10.0]])
    out = tmp_path / "p.md"
    subprocess.run([sys.executable, "-m", "paper_2112_00821_amd.profsum", "--trace", str(tmp_path / "trace"),
                    "--fetch", str(tmp_path / "FETCH_SIZE"), "--write", str(tmp_path / "WRITE_SIZE"),
                    "--copy-mb", str(mb), "--kernel", "k_sweep", "--workload", "synthetic", "--out", str(out)],
                   check=True, cwd=ROOT)
    rec = profsum.read_traffic(str(out), "k_sweep")
    assert rec["fetch_bytes_per_launch"] == pytest.approx((600 + 300 + 30) / 3 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx((900 + 450 + 60) / 3 * 1024 * 1.0)
    assert rec["instantiation"] == "k_sweep<9, 7, 8, false, 0>"
    assert sorted(rec["instantiations"]) == ["k_sweep<9, 7, 4, false, 0>", "k_sweep<9, 7, 8, false, 0>"]
