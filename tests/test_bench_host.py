"""Host-side logic of the benchmark, on the CPU: the algorithmic bytes of a
Jacobi sweep, the fields of the oracle baseline, and the one-GPU limit."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1908_01762_amd import cases  # noqa: E402


def test_sweep_bytes_rows_and_pairs():
    # 100 rows, 1,600 slots = 100 self slots + 1,500 stored pairs
    mixed = cases.taylor_green(10, precision="mixed")
    b = bench.sweep_bytes(mixed, slots=1600, index_bits=16)
    # row: count 4, RHS 8, D_ii 8, flag 4, own p 8, new p 8, new p32 4, gathered p32 4
    assert (b["per_row"], b["per_pair"], b["pairs"]) == (48, 6, 1500)
    assert b["bytes"] == 100 * 48 + 1500 * 6
    assert b["wall_rows"] == 0 and b["per_wall_row"] == 0
    fp64 = cases.taylor_green(10, precision="fp64")
    b = bench.sweep_bytes(fp64, slots=1600)
    assert (b["per_row"], b["per_pair"]) == (48, 12)
    assert b["bytes"] == 100 * 48 + 1500 * 12


def test_sweep_bytes_walls():
    mixed = cases.taylor_green(10, precision="mixed")
    b = bench.sweep_bytes(mixed, slots=1600, index_bits=32, wall_pairs=300, wall_rows=20)
    # wall row: count 4, hydrostatic term 8, new p 8, its FP32 copy 4; wall pair: weight + index
    assert (b["per_wall_row"], b["per_wall_pair"]) == (24, 8)
    assert b["bytes"] == 100 * 48 + 1500 * 8 and b["wall_bytes"] == 20 * 24 + 300 * 8
    packed = bench.sweep_bytes(mixed, slots=1600, index_bits=12)
    assert packed["per_row"] == 36 and packed["per_pair"] == 5.5
    assert packed["bytes"] == 100 * 36 + 1500 * 5.5
    fp64 = cases.taylor_green(10, precision="fp64")
    b = bench.sweep_bytes(fp64, slots=1600, wall_pairs=300, wall_rows=20)
    assert (b["per_wall_row"], b["per_wall_pair"]) == (20, 12)


def test_unit_bytes_of_the_cached_coefficient_sweep():
    # coefficients over the lattice neighbours (self excluded), bitmask over
    # the stencil candidates, 40 B of per-particle data
    assert bench.UNIT_BYTES[(3, "mixed")] == 420
    assert bench.UNIT_BYTES[(2, "mixed")] == 128
    assert bench.UNIT_BYTES[(2, "fp64")] == 208
    assert bench.UNIT_BYTES[(3, "fp64")] == 740


def test_cpu_baseline_fields():
    import oracle
    c = cases.taylor_green(10)
    out = bench.cpu_baseline(c, budget_s=0.0)   # one oracle step
    assert out["kind"] == "oracle" and out["unit"] == "particle-iters/s"
    assert out["cores"] == oracle.threads(parallel=True) >= 1
    assert out["value"] > 0 and out["particle_steps_per_s"] > 0
    assert "first 1 step(s)" in out["sample"]
    host = out["host"]
    assert host["nproc"] >= 1 and set(host) == {"nproc", "usable_cpus", "cpu_model"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
