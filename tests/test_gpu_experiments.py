"""Solver-variant harnesses on the GPU (short runs): the tolerance sweep and
EISPH (one forced sweep per step) against SISPH."""
import pytest

from paper_1908_01762_amd import experiments

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tolerance_sweep_monotone_in_sweeps():
    _gpu()
    rows = experiments.tolerance_sweep(n=40, steps=10, tolerances=(0.1, 1e-2, 1e-3))
    print(rows, flush=True)
    sweeps = [r["mean_sweeps"] for r in rows]
    assert sweeps[0] <= sweeps[1] <= sweeps[2]
    assert all(r["decay_error_max"] < 0.05 for r in rows)


def test_eisph_runs_one_sweep_per_step():
    _gpu()
    r = experiments.eisph_vs_sisph(n=40, steps=10)
    print(r, flush=True)
    assert r["eisph"]["mean_sweeps"] == 1.0 and r["eisph"]["max_sweeps"] == 1
    assert r["sisph"]["mean_sweeps"] >= 2.0
