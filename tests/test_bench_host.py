"""Host-side logic of bench.py: the one-GPU guard, the source-keyed HBM traffic
record and the device-memory BP roofline (no GPU needed)."""
import hashlib
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "only one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_valid_only_for_its_sources(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("__global__ void k() {}\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    monkeypatch.setattr(bench, "TRAFFIC", {"w": {"k": {"src": [str(src)], "sha256": digest,
                                                       "fetch_kib": 100.0, "write_kib": 50.0}}})
    want = (100.0 * bench.FETCH_SCALE + 50.0 * bench.WRITE_SCALE) * 1024.0
    assert bench.traffic_bytes("w", "k") == pytest.approx(want)
    assert abs(bench.FETCH_SCALE - 2.0) < 1e-3 and bench.WRITE_SCALE == 1.0   # 1 GiB copy calibration
    assert bench.traffic_bytes("w", "other") is None and bench.traffic_bytes("x", "k") is None
    src.write_text("__global__ void k() { }\n")                   # the kernel changed since the counters
    assert bench.traffic_bytes("w", "k") is None


def test_device_state_roofline_counts_state_once_per_iteration():
    small = SimpleNamespace(rows=10, cols=50, edges=101)
    large = SimpleNamespace(rows=1000, cols=6000, edges=12003)
    # (dem, stats, shots, state in device memory)
    parts = [(small, {"bp_iters": 700}, 64, False), (large, {"bp_iters": 900}, 64, True),
             (large, {"bp_iters": 300}, 64, True)]
    kern = {"k_bp_dev": (4, 8.0), "k_bp": (4, 1.0), "k_osd": (4, 2.0)}   # (launches, total ms)
    r = bench.roofline(kern, parts, [])
    per_shot_iter = 16 * (1000 + 1) + 4 * 6000 + 12004                  # checks (+1 pad), columns, edge bytes
    byts = 2 * per_shot_iter * (900 + 300)                                # read and written once
    assert r["kernel"] == "k_bp_dev" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["avg_launch_ms"] == pytest.approx(2.0) and r["launches"] == 4
    assert r["achieved"] == pytest.approx(byts / 8e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
