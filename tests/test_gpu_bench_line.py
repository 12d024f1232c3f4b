"""The benchmark's JSON line on the GPU, from a short run of bench.py in a
child process: every field the line promises, with consistent values."""
import json
import math
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
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
           "--secondary-steps", "3", "--no-batch-compare", "--no-serving", "--no-solver-compare",
           "--cpu-budget", "0.1"]
    print("running", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=400)
    print(r.stderr[-3000:], flush=True)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "secondary"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "particle-iters/s" and d["data"] == "synthetic" and d["dtype"] == "f32+f64"
    assert d["config"]["workload"] == "db3d_dx0.01_mixed" and d["config"]["launch"] == "eager"
    assert d["config"]["fluid_particles"] == 2000000 and d["config"]["wall_particles"] == 1343508
    rf = d["roofline"]
    print("roofline", rf, flush=True)
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] > 0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    # achieved = 420 B per fluid particle and effective sweep / sweep-kernel time
    assert rf["algorithmic_bytes_per_particle_iter"] == 420
    assert rf["algorithmic_bytes_per_sweep"] == 420 * 2000000
    per_launch = rf["algorithmic_bytes_per_launch"] / (rf["avg_launch_us"] * 1e-6) / 1e9
    assert abs(per_launch - rf["achieved"]) < 0.01 * rf["achieved"]
    # walls: per-sweep launches, each timed on its own, the wall pass apart
    assert rf["mode"] == "per-sweep launches" and rf["persistent_launches"] == 0
    assert rf["launches"] == rf["per_sweep_launches"] >= rf["effective_sweeps"] > 0
    # every eighth launch of a solve timed (launch 0 of every solve among them)
    assert rf["timing_period"] == 8 and 0 < rf["timed_launches"] <= rf["launches"]
    assert rf["timed_launches"] >= rf["launches"] // 8
    # chunk time less the sweep kernel's (sampled) time, per launch: the wall
    # pass and the launch gaps; on a two-step run the sampling noise of the
    # sweep average is of the same size, so only its presence is checked
    assert rf["wall_pass"]["rows"] > 0 and math.isfinite(rf["wall_pass"]["us_per_sweep"])
    assert rf["layout"]["bytes_per_sweep"] > 0
    # the counter-measured bytes and their rate, when the committed counter
    # summary was taken on the current kernel source
    if rf["traffic"] is not None:
        assert rf["traffic"] > 0 and abs(rf["traffic_frac"] - rf["traffic_GBps"] / rf["peak"]) < 1e-3
    # the plain-read probe of 1 GiB, and the kernel's rate against it
    big = [c for c in d["copy_reference"] if c["mib"] == 1024][0]
    assert 0 < big["read_GBps"] < rf["peak"] and rf["read_probe_GBps"] == big["read_GBps"]
    assert abs(rf["frac_of_read_probe"] - rf["achieved"] / big["read_GBps"]) < 1e-3
    assert d["gtvf_short_lists_last_step"] == 1   # the dam break's sub-steps walked the short lists
    sec = d["secondary"]
    assert sec["config"]["workload"] == "tg400_wendland_mixed"
    sr = sec["roofline"]
    assert sr["algorithmic_bytes_per_particle_iter"] == 128
    assert sr["launches"] == sr["persistent_launches"] + sr["per_sweep_launches"]
    assert sr["timing_period"] == 1 and sr["timed_launches"] == sr["launches"]
    # one persistent launch per solve unless the runtime refused one (for
    # instance while another process holds the device), which is counted
    if sr["per_sweep_launches"]:
        assert sr["persistent_fallbacks"]["refused"] + sr["persistent_fallbacks"]["timed_out"] > 0
    else:
        assert sr["mode"] == "persistent" and sr["persistent_launches"] == 3
    assert sec["solves_at_max_iter"] == 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["unit"] == d["unit"]
    assert cb["host"]["nproc"] >= 1
