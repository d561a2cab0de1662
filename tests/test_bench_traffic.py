"""The measured-traffic figure bench.py reports for the trace kernel: the
committed counter summary is self-consistent (traffic = FETCH_SIZE and
WRITE_SIZE in KiB times their copy-calibrated factors; algorithmic bytes =
queries x B(M) at the theater's 436,120 triangles), and the figure is withheld
(None) once the kernel source differs from the one the counters were taken on."""
import os
import re
import shutil

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COUNTERS = os.path.join(ROOT, "profiles", "k_trace_theater_436k_counters.txt")


def _kv(path):
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    return kv


def test_counter_summary_is_self_consistent():
    kv = _kv(COUNTERS)
    traffic = (float(kv["fetch_size_kib"]) * float(kv["fetch_scale"])
               + float(kv["write_size_kib"]) * float(kv["write_scale"])) * 1024
    # the KiB figures are printed to 0.1 KiB
    assert abs(traffic - int(kv["traffic_bytes_per_launch"])) <= 0.05 * 1024 * 2 + 1
    # queries per launch, as the summary's header states them
    q = int(re.search(r"([\d,]+) queries", open(COUNTERS).read()).group(1).replace(",", ""))
    assert bench.algorithmic_bytes_per_query(436_120) == 1028
    assert int(kv["algorithmic_bytes_per_launch"]) == q * 1028


def test_traffic_withheld_when_kernel_source_changes(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    os.makedirs(tmp_path / "paper_1811_05784_amd" / "csrc")
    shutil.copy(COUNTERS, tmp_path / "profiles")
    src = os.path.join(ROOT, "paper_1811_05784_amd", "csrc", "trace.hip")
    dst = tmp_path / "paper_1811_05784_amd" / "csrc" / "trace.hip"
    shutil.copy(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    same = bench.measured_traffic()
    with open(dst, "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic() is None
    # the committed tree: the figure is reported exactly when the sources agree
    monkeypatch.setattr(bench, "ROOT", ROOT)
    assert bench.measured_traffic() == same
    if same is not None:
        assert same == int(_kv(COUNTERS)["traffic_bytes_per_launch"])
