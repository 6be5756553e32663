"""The benchmark's command-line contract: one JSON line with the metric, the whole-job
value, the roofline of the dominant kernel and the configuration; more than one GPU is
refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_prints_one_json_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "droplet64", "--steps",
                        "40", "--warmup", "4", "--no-cpu-baseline", "--sample-every", "10"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 40 and d["warmup"] == 4 and d["value"] > 0
    assert d["unit"] == "MLUPS" and d["dtype"] == "f64" and d["config"]["workload"].startswith("droplet-64x64")
    roof = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in roof, key
    assert roof["kernel"] in ("mag", "stage1", "stage2", "stage3") and 0 < roof["frac"] < 1
    assert roof["peak"] == (78.6 if roof["bound"] == "alu" else 8000.0)   # FP64 vector peak, HBM
    assert roof["timed_launches"] == 4
