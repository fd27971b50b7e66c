"""bench.py end to end on a small workload: one JSON line with the fields
the measurement contract names (metric, value, roofline, per-precision
results, the opt-in fused steps), every rate positive."""
import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT

pytestmark = pytest.mark.gpu


def test_bench_prints_one_complete_json_line():
    print("bench.py --workload adv2d_16", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "adv2d_16", "--steps", "3",
                        "--warmup", "1", "--reps", "2", "--no-cpu"], capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "precisions", "fused"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 3 and out["warmup"] == 1 and out["value"] > 0
    assert out["config"]["workload"].startswith("adv2d_16")
    roof = out["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] == "hbm" and roof["peak"] == 8000.0 and roof["achieved"] > 0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    assert set(out["precisions"]) == {"fp32refine48", "fp64", "fp32refine", "fp32"}
    for p, e in out["precisions"].items():
        assert e["value"] > 0 and e["sweep_us"] > 0 and e["relax_us"] > 0, p
    for p in ("fp32refine48", "fp64"):
        assert out["fused"][p]["value"] > 0 and out["fused"][p]["vs_separate_passes"] > 0
