"""Host logic of the benchmark: the one-GPU contract, the algorithmic byte
model of the passes, and when the committed counter summary is used."""
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_pass_bytes_embryo_model():
    """512x512x256, six 31x31x41 PSFs, weights: 8.03 B/voxel per y pass,
    8.03 + 0.64 per z pass, 12.03 for the ratio and 20.03 for the update
    pass; 81.54 B/voxel per view-update (8 passes)."""
    blk = SimpleNamespace(dims=(512, 512, 256), psfs=[np.zeros((41, 31, 31))] * 6)
    by = bench.pass_bytes([blk], True)
    V = 512 * 512 * 256
    per = {k: v / V for k, v in by.items()}
    assert abs(per["y_forward"] - 8.031) < 1e-3 and per["y_inverse"] == per["y_forward"]
    assert abs(per["z_product"] - per["y_forward"] - 41 * 257 * 8 / (512 * 256)) < 1e-9  # 0.643
    assert abs(per["x_ratio"] - (per["y_forward"] + 4)) < 1e-9
    assert abs(per["x_update"] - (per["y_forward"] + 12)) < 1e-9
    total = 2 * (per["y_forward"] + per["z_product"] + per["y_inverse"]) + per["x_ratio"] + per["x_update"]
    assert abs(total - 81.54) < 0.01
    assert abs(bench.pass_bytes([blk], False)["x_update"] / V - (per["y_forward"] + 8)) < 1e-9


def test_measured_traffic_only_for_the_profiled_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "hbm_traffic_embryo512.txt")
    txt = open(path).read()
    h = txt.split("source_hash:")[1].split()[0]
    monkeypatch.setattr(bench, "source_hash", lambda: h)
    t = bench.measured_traffic("embryo512", "z_product")
    assert t is not None and t > 0
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("embryo512", "z_product") is None
    assert bench.measured_traffic("no_such_workload", "z_product") is None
