"""The benchmark's JSON line on the GPU, from a short run of bench.py in a
child process: every field the line promises, with consistent values."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_fields():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "2",
           "--no-batch-compare", "--no-serving", "--no-solver-compare", "--cpu-budget", "0.1"]
    print("running", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    print(r.stderr[-3000:], flush=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 2
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "particle-iters/s" and d["data"] == "synthetic" and d["dtype"] == "f32+f64"
    assert d["config"]["workload"] == "tg400_wendland_mixed" and d["config"]["launch"] == "eager"
    rf = d["roofline"]
    print("roofline", {k: v for k, v in rf.items() if k != "kernel"}, flush=True)
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] > 0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["sweeps"] >= rf["effective_sweeps"] > 0
    # one launch per solve, or (the cooperative launch refused, e.g. while
    # another process holds the device) one per sweep, with the fallback counted
    if rf["mode"] == "persistent":
        assert rf["launches"] == 3
    else:
        assert rf["launches"] == rf["sweeps"]
        assert rf["persistent_fallbacks"]["refused"] + rf["persistent_fallbacks"]["timed_out"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["unit"] == d["unit"]
    assert cb["host"]["nproc"] >= 1
