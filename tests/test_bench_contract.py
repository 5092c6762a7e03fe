"""Host-side parts of the benchmark contract (no GPU): the one-GPU guard and
the reading of the committed HBM traffic passes."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """--gpus above 1 prints one JSON line naming the one-GPU limit and exits
    before touching a device"""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _traffic_file(tmp_path, src_hash):
    p = tmp_path / "traffic.txt"
    p.write_text("# comment line\n"
                 f"source_hash {src_hash}\n"
                 "fetch_scale 2.0\n"
                 "write_scale 1.0\n"
                 "config 4 4 100.0 300.0\n"
                 "config 2 8 10.0 20.0\n")
    return str(p)


def test_traffic_is_scaled_fetch_plus_write(tmp_path, monkeypatch):
    """bytes per launch = 1024 * (FETCH_SIZE * fetch_scale + WRITE_SIZE *
    write_scale), per launch configuration"""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, "abc"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.profiled_traffic(4, 4) == 1024.0 * (100.0 * 2.0 + 300.0 * 1.0)
    assert bench.profiled_traffic(2, 8) == 1024.0 * (10.0 * 2.0 + 20.0 * 1.0)
    assert bench.profiled_traffic(8, 8) is None  # configuration not profiled


def test_traffic_is_dropped_once_the_kernel_changed(tmp_path, monkeypatch):
    """counters taken on other kernel sources are not reported"""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, "abc"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.profiled_traffic(4, 4) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.profiled_traffic(4, 4) is None


def test_committed_traffic_file_parses():
    """the committed passes cover the tuned configurations of the 2D FP64
    kernel; while their source hash matches, each gives 1.0-1.2x the 1.07 GB
    of algorithmic traffic of one launch"""
    if bench.profiled_traffic(4, 4) is None:
        pytest.skip("kernel sources changed since the counter passes were taken")
    alg = 16.0 * 256 * 256 * 1024
    for cfg in ((4, 4), (2, 4), (4, 8), (2, 8)):
        t = bench.profiled_traffic(*cfg)
        assert t is not None and 1.0 <= t / alg <= 1.2, (cfg, t)
