"""The benchmark's output contract: one JSON line with the metric, the
whole-job value, the roofline object (achieved bytes over the measured time
against the HBM peak) and the CPU-baseline slot, from a short run of the
real script in a child process (headline only, no probes or workloads)."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
                          "--no-variants", "--no-configs", "--no-cpu", "--no-copy"],
                         capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["unit"] == "GLUP/s"
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    # value and achieved are the same measurement in two units
    lups = d["config"]["rows"] * d["config"]["nb"]
    assert abs(d["value"] - lups / (d["ms_per_step"] * 1e-3) / 1e9) < 1e-2 * d["value"]
    assert abs(r["achieved"] - r["bytes_per_launch"] / (d["ms_per_step"] * 1e-3) / 1e9) < 1e-2 * r["achieved"]
