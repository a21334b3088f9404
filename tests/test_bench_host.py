"""Host-side checks of bench.py (no GPU): the one-GPU contract, and the
hardware-counter traffic record it reports beside the render's roofline."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_consistent():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    cal = rec["copy_calibration"]
    # the scale factors are the copy kernel's true bytes over its counter bytes
    assert abs(cal["fetch_scale"] - cal["bytes_read"] / (cal["FETCH_SIZE_KiB"] * 1024)) < 1e-9
    assert abs(cal["write_scale"] - cal["bytes_written"] / (cal["WRITE_SIZE_KiB"] * 1024)) < 1e-9
    fetch = np.mean(rec["render_FETCH_SIZE_KiB"]) * 1024 * cal["fetch_scale"]
    write = np.mean(rec["render_WRITE_SIZE_KiB"]) * 1024 * cal["write_scale"]
    assert abs(fetch - rec["fetch_bytes_per_launch"]) <= 1e-6 * fetch
    assert abs(write - rec["write_bytes_per_launch"]) <= 1e-6 * write
    assert abs(fetch + write - rec["bytes_per_launch"]) <= 1e-6 * (fetch + write)
    # algorithmic bytes: the unconvolved C1 images plus the per-point constants
    assert rec["algorithmic_bytes_per_launch"] == 4096 * 200 * 200 * 4 + 4096 * 2304
    # the commands run committed files only, with the program right after --
    for cmd in rec["commands"].values():
        assert "-- python3 bench.py" in cmd and "_work" not in cmd


def test_traffic_is_withheld_when_the_render_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "render_sources_digest", lambda: "0" * 64)
    assert bench.measured_traffic() is None
