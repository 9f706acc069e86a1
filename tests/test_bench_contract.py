"""The benchmark's host-side contract (no GPU): the byte model the roofline prices the
raster kernels with, the guard that drops measured traffic taken with other kernel
sources or another workload, and the single-GPU refusal of --gpus N > 1."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_raster_byte_model():
    P, K = 87_584_665, 209_978_602            # c3: pixels, (tile, surfel) pairs
    # backward: 68 bytes per pixel, record re-read (72) + record gradient (64) per pair
    assert bench.raster_kernel_bytes("raster_bwd", P, K) == 68 * P + 136 * K == 34_512_847_092
    # forward: record (72) per pair, 52 bytes of outputs per pixel
    assert bench.raster_kernel_bytes("raster_fwd", P, K) == 72 * K + 52 * P


def test_measured_traffic_needs_matching_sources_and_workload(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    rel = os.path.relpath(src, bench.ROOT)
    rec = {"workload": "w", "tile": 8, "batch_depth": 64, "source_files": [rel],
           "source_sha256": bench.kernel_source_digest([rel]),
           "kernels": {"raster_bwd": {"bytes_per_launch": 123}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(path))
    assert bench.measured_traffic("raster_bwd", "w", 8, 64) == 123
    assert bench.measured_traffic("raster_fwd", "w", 8, 64) is None        # not recorded
    assert bench.measured_traffic("raster_bwd", "w", 16, 64) is None       # other tile
    assert bench.measured_traffic("raster_bwd", "other", 8, 64) is None    # other workload
    src.write_text("kernel v2\n")                                         # sources changed
    assert bench.measured_traffic("raster_bwd", "w", 8, 64) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
