"""Scheduling logic of the continuous-batching loop, on the CPU, against a
stand-in backend and a fake clock: admission by workspace bytes and slots,
arrival order, joining while others run, eviction of a failing case and the
latency bookkeeping."""
import dataclasses

import numpy as np

from paper_1908_01762_amd.serve import Request, Server


@dataclasses.dataclass
class FakeCase:
    n_fluid: int
    fail_at: int = -1


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeBackend:
    """Workspace = 100 B per particle; a batched step costs 1 us per particle."""

    def __init__(self, clock):
        self.clock = clock
        self.steps_of = {}
        self.resident = set()
        self.max_resident = 0
        self.log = []

    def workspace_bytes(self, case):
        return 100 * case.n_fluid

    def admit(self, case):
        h = object()
        self.steps_of[h] = (case, 0)
        self.resident.add(h)
        self.max_resident = max(self.max_resident, len(self.resident))
        self.log.append(("admit", self.clock(), case.n_fluid))
        return h

    def step(self, handles):
        self.clock.t += 1e-6 * sum(self.steps_of[h][0].n_fluid for h in handles)
        out = []
        for h in handles:
            case, n = self.steps_of[h]
            self.steps_of[h] = (case, n + 1)
            if n == case.fail_at:
                out.append({"iters": 0, "error": "non-finite pressure"})
            else:
                out.append({"iters": 3})
        return out

    def release(self, h, keep_result):
        self.resident.discard(h)
        return self.steps_of[h][1] if keep_result else None

    def sync(self):
        pass


def run(reqs, budget, slots):
    clock = Clock()
    be = FakeBackend(clock)
    srv = Server(be, budget_bytes=budget, max_slots=slots, clock=clock, sleep=clock.sleep)
    rep = srv.run(reqs)
    return srv, be, rep


def test_all_requests_complete_with_their_step_counts():
    reqs = [Request(k, arrival=0.01 * k, case=FakeCase(1000 + 100 * k), steps=5 + k % 3) for k in range(12)]
    srv, be, rep = run(reqs, budget=10**9, slots=64)
    assert rep["completed"] == 12 and rep["failed"] == 0
    for r in srv.done:
        assert r.steps_done == r.steps and r.result == r.steps
        assert r.admitted >= r.arrival and r.finished >= r.admitted


def test_admission_respects_bytes_slots_and_arrival_order():
    reqs = [Request(k, arrival=0.0, case=FakeCase(1000), steps=4) for k in range(6)]
    # budget fits two cases (200 kB), slots allow three
    srv, be, rep = run(reqs, budget=250_000, slots=3)
    assert be.max_resident == 2
    assert rep["peak_resident_bytes"] <= 250_000
    order = [r.rid for r in sorted(srv.done, key=lambda r: (r.admitted, r.rid))]
    assert order == sorted(order)
    srv, be, rep = run([Request(k, 0.0, FakeCase(10), 4) for k in range(6)], budget=10**9, slots=3)
    assert be.max_resident == 3


def test_oversized_request_is_rejected_others_run():
    reqs = [Request(0, 0.0, FakeCase(100), 3), Request(1, 0.0, FakeCase(10**6), 3),
            Request(2, 0.0, FakeCase(100), 3)]
    srv, be, rep = run(reqs, budget=50_000, slots=8)
    assert rep["failed"] == 1 and rep["completed"] == 2
    bad = [r for r in srv.done if r.error][0]
    assert bad.rid == 1 and "exceeds the budget" in bad.error


def test_late_arrival_joins_running_batch():
    reqs = [Request(0, 0.0, FakeCase(10_000), 50), Request(1, 0.05, FakeCase(10_000), 5)]
    srv, be, rep = run(reqs, budget=10**9, slots=8)
    r0, r1 = sorted(srv.done, key=lambda r: r.rid)
    assert r1.admitted < r0.finished          # joined while request 0 was running
    assert r1.finished < r0.finished
    assert rep["max_batch_size"] == 2


def test_failing_case_is_evicted_without_stopping_others():
    reqs = [Request(0, 0.0, FakeCase(500, fail_at=2), 10), Request(1, 0.0, FakeCase(500), 10)]
    srv, be, rep = run(reqs, budget=10**9, slots=8)
    r0, r1 = sorted(srv.done, key=lambda r: r.rid)
    assert r0.error and r0.steps_done == 2 and r0.result is None
    assert not r1.error and r1.steps_done == 10
    assert rep["failed"] == 1


def test_latency_percentiles_match_the_recorded_steps():
    reqs = [Request(k, 0.0, FakeCase(1000 * (k + 1)), 3) for k in range(4)]
    srv, be, rep = run(reqs, budget=10**9, slots=8)
    steps = np.array(srv.step_ms)
    assert len(steps) == 3
    # every step holds all four cases: 10,000 particles -> 10 ms
    assert np.allclose(steps, 10.0)
    assert abs(rep["p99_step_ms"] - 10.0) < 1e-9 and abs(rep["p50_step_ms"] - 10.0) < 1e-9
    assert rep["particle_steps_per_s"] > 0
