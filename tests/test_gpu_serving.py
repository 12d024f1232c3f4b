"""Serving on the GPU: requests arrive over time, are admitted by workspace
bytes into one batch, run while others join and leave, and each result is
bitwise the state the same case reaches when run alone."""
import numpy as np
import pytest

from paper_1908_01762_amd import cases
from paper_1908_01762_amd.serve import GpuBackend, Request, Server

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01762_amd import sisph
    return sisph


def test_serving_results_equal_solo_runs():
    sisph = _gpu()
    mix = cases.serving_mix(n_cases=10, seed=5, rate_hz=200.0, n_min=300, n_max=3000)
    reqs = [Request(k, t, c, steps=4 + (k % 3)) for k, (t, c) in enumerate(mix)]
    budget = int(3.5 * max(sisph.workspace_bytes(c) for _, c in mix))
    backend = GpuBackend(max_slots=6)
    srv = Server(backend, budget_bytes=budget, max_slots=6)
    rep = srv.run(reqs)
    print(rep, flush=True)
    assert rep["completed"] == len(reqs) and rep["failed"] == 0
    assert rep["max_batch_size"] >= 2
    assert rep["peak_resident_bytes"] <= budget
    for r in srv.done:
        ctx = sisph.Context(r.case)
        ctx.step(r.steps)
        solo = ctx.read_state()
        ctx.close()
        for k in ("x", "u", "ut", "p"):
            assert np.array_equal(r.result[k], solo[k]), (r.rid, k)
    backend.close()
