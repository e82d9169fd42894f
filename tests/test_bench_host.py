"""Host logic of bench.py (no GPU): the one-GPU guard, the CPU-baseline
fields, and the rule that counter summaries count only for the kernel
sources they were measured with."""
import os
import subprocess
import sys

import bench
from paper_2510_11527_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_all_cores_and_one_core():
    items = W.config4(n_inst=3, sizes=(16, 24))
    cb = bench.cpu_baseline(items, 500)
    assert cb["kind"] == "oracle" and cb["unit"] == bench.UNIT
    assert cb["value"] > 0 and cb["cores"] >= 1 and "instances" in cb["sample"]
    one = cb["single_core"]
    assert one["cores"] == 1 and one["value"] > 0 and "forward-Euler" in one["sample"]


def test_counter_summaries_count_only_for_their_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_w_traffic.txt").write_text(
        "# header\nsource_sha=abc\ntile=t1\nworkload=w1\ntraffic_bytes_per_launch=123\nvalu_busy_pct=45.5\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "abc")
    assert bench.measured_traffic("w1", "t1") == 123.0
    assert bench.measured_valu_busy("w1", "t1") == 45.5
    assert bench.measured_traffic("w1", "t2") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "other")
    assert bench.measured_traffic("w1", "t1") is None
    assert bench.measured_valu_busy("w1", "t1") is None
