"""bench.py's one-line JSON record on a small workload: the fields a reader
of the record relies on, with a live roofline block (GPU)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_record_on_the_small_vortex_mesh():
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "vortex",
                          "--steps", "20", "--warmup", "2", "--no-fp64", "--no-cpu-baseline"],
                         cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [l for l in out.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["steps"] == 20 and rec["warmup"] == 2
    assert rec["value"] > 0 and rec["dtype"] == "f32" and rec["higher_is_better"] is True
    assert rec["config"]["P"] == 2 and rec["config"]["K"] > 0
    r = rec["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert r["launches"] == 5 * 20 and r["avg_launch_us"] > 0
    # value and the launch time describe the same run: DOF x 5 stages per step
    dof = rec["config"]["dof"]
    assert abs(rec["value"] * rec["ms_per_step"] * 1e-3 - dof * 5) / (dof * 5) < 1e-6
