"""bench.py end to end on a small block (256^3, a few steps, no adjoint,
paper-block or CPU legs): one JSON line on stdout carrying the contract's
fields, the roofline object and the FP64 and FP16 legs."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "256", "--steps", "4", "--warmup", "2",
           "--fp64-steps", "2", "--fp16-steps", "2", "--no-adjoint", "--no-paper-block", "--no-cpu-baseline"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    line = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 4 and line["warmup"] == 2
    assert line["value"] > 0 and line["higher_is_better"] is True
    assert "workload" in line["config"]
    roof = line["roofline"]
    assert roof["bound"] == "hbm" and roof["peak"] == 8000.0 and roof["unit"] == "GB/s"
    assert 0.0 < roof["frac"] < 1.0 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert roof["algorithmic_bytes_per_cell"] == 452.0
    for leg, bpc in (("fp64", 904.0), ("fp16", 364.0)):
        assert line[leg]["value"] > 0
        assert line[leg]["roofline"]["algorithmic_bytes_per_cell"] == bpc
