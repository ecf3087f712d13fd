"""bench.py's command-line contract, checked without a GPU: the multi-GPU
invocation is refused with a message (one GPU is the unit measured), and the
roofline object is built from the scope table's per-cell bytes with the fused
kernel's own minimum beside it."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_object():
    sys.path.insert(0, ROOT)
    import bench
    ncell = 512 ** 3
    ms = 11.4
    res = {"kernels": {"step": {"avg_ms": ms, "algorithmic_bytes_per_launch": 432.0 * ncell,
                                "achieved_GBs": 432.0 * ncell / (ms * 1e-3) / 1e9}},
           "step_bytes_per_cell": 432.0, "ncell": ncell}
    r = bench.roofline(res, "fp32")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["algorithmic_bytes_per_cell"] == 452.0
    assert abs(r["achieved"] - 452.0 * ncell / (ms * 1e-3) / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert r["fused_kernel_min_bytes_per_cell"] == 432.0
    assert r["fused_kernel_min_frac"] < r["frac"]
    for prec, b in (("fp64", 904.0), ("fp16", 364.0)):
        assert bench.roofline(res, prec)["algorithmic_bytes_per_cell"] == b
