"""Continuous-batching request loop for independent SISPH cases.

Requests (a case and a number of steps) arrive over time.  A request is
admitted when a batch slot is free and its device workspace fits the HBM
budget; admitted cases stay resident on the GPU and are stepped together,
one batched launch per kernel per step.  A request that arrives while
others are running joins at the next step boundary; a finished case leaves
and frees its memory and slot, which may admit queued requests.  The loop
records the latency of every batched step, per-request latency and the
throughput.

Scheduling only: all compute is the library's batched step.  The backend
is an object with the methods used below; ``GpuBackend`` drives libsisph,
tests may pass a stand-in with a fake clock.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    case: Any
    steps: int
    admitted: Optional[float] = None
    finished: Optional[float] = None
    steps_done: int = 0
    ppe_iters: int = 0
    handle: Any = None
    result: Any = None
    error: Optional[str] = None


class GpuBackend:
    """libsisph: one Context per admitted case, one Batch for all of them."""

    def __init__(self, max_slots: int):
        import torch
        from . import sisph
        self.sisph = sisph
        self.torch = torch
        self.batch = sisph.Batch(max_slots)
        self.batch.use_graphs(True)   # fixed step segments replayed from HIP graphs

    def workspace_bytes(self, case) -> int:
        return self.sisph.workspace_bytes(case)

    def admit(self, case):
        ctx = self.sisph.Context(case, stream=self.batch.stream)
        self.batch.attach(ctx)
        return ctx

    def step(self, handles) -> List[dict]:
        out = self.batch.step(raise_on_error=False)
        for s, h in zip(out, handles):
            if s["case_status"] < 0:
                s["error"] = self.sisph.lib().sisph_last_error(h.h).decode() or \
                    self.sisph.status_string(s["case_status"])
        return out

    def release(self, handle, keep_result: bool):
        res = handle.read_state() if keep_result else None
        self.batch.detach(handle)
        handle.close()
        handle.workspace = None
        return res

    def sync(self):
        self.torch.cuda.synchronize()

    def close(self):
        self.batch.close()


class Server:
    def __init__(self, backend, budget_bytes: int, max_slots: int,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, keep_results: bool = True):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.sleep = sleep
        self.keep_results = keep_results
        self.queue: deque = deque()
        self.resident: List[Request] = []
        self.done: List[Request] = []
        self.resident_bytes = 0
        self.step_ms: List[float] = []
        self.batch_sizes: List[int] = []
        self.peak_bytes = 0
        self.t0 = 0.0

    # ---------------------------------------------------------------- steps
    def _admit(self, now: float):
        while self.queue and self.queue[0].arrival <= now and len(self.resident) < self.max_slots:
            r = self.queue[0]
            need = self.backend.workspace_bytes(r.case)
            if need > self.budget:
                self.queue.popleft()
                r.error = f"workspace {need} B exceeds the budget {self.budget} B"
                r.finished = now
                self.done.append(r)
                continue
            if self.resident_bytes + need > self.budget:
                break   # wait for memory: keep arrival order
            self.queue.popleft()
            r.handle = self.backend.admit(r.case)
            r.admitted = now
            self.resident.append(r)
            self.resident_bytes += need
            self.peak_bytes = max(self.peak_bytes, self.resident_bytes)

    def _retire(self, now: float):
        keep = []
        for r in self.resident:
            if r.steps_done >= r.steps or r.error:
                r.result = self.backend.release(r.handle, self.keep_results and not r.error)
                r.handle = None
                r.finished = now
                self.resident_bytes -= self.backend.workspace_bytes(r.case)
                self.done.append(r)
            else:
                keep.append(r)
        self.resident = keep

    def run(self, requests: List[Request]) -> Dict[str, Any]:
        self.queue = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        self.t0 = self.clock()
        total = len(self.queue)
        while len(self.done) < total:
            now = self.clock() - self.t0
            self._admit(now)
            if not self.resident:
                if self.queue:
                    wait = self.queue[0].arrival - now
                    if wait > 0:
                        self.sleep(wait)
                continue
            t = self.clock()
            stats = self.backend.step([r.handle for r in self.resident])
            self.backend.sync()
            dt = self.clock() - t
            self.step_ms.append(dt * 1e3)
            self.batch_sizes.append(len(self.resident))
            for r, s in zip(self.resident, stats):
                if s.get("error"):
                    r.error = s["error"]
                    continue
                r.steps_done += 1
                r.ppe_iters += int(s["iters"])
            self._retire(self.clock() - self.t0)
        return self.report()

    # --------------------------------------------------------------- report
    def report(self) -> Dict[str, Any]:
        ok = [r for r in self.done if not r.error]
        wall = max((r.finished for r in self.done), default=0.0)
        steps = np.array(self.step_ms) if self.step_ms else np.zeros(1)
        lat = np.array([r.finished - r.arrival for r in ok]) if ok else np.zeros(1)
        wait = np.array([r.admitted - r.arrival for r in ok]) if ok else np.zeros(1)
        particle_steps = sum(r.case.n_fluid * r.steps_done for r in ok)
        ppe = sum(r.case.n_fluid * r.ppe_iters for r in ok)
        return {
            "requests": len(self.done),
            "completed": len(ok),
            "failed": len(self.done) - len(ok),
            "batched_steps": len(self.step_ms),
            "mean_batch_size": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "max_batch_size": int(max(self.batch_sizes)) if self.batch_sizes else 0,
            "p50_step_ms": float(np.percentile(steps, 50)),
            "p99_step_ms": float(np.percentile(steps, 99)),
            "p50_request_s": float(np.percentile(lat, 50)),
            "p99_request_s": float(np.percentile(lat, 99)),
            "p99_queue_wait_s": float(np.percentile(wait, 99)),
            "wall_s": wall,
            "particle_steps_per_s": particle_steps / wall if wall > 0 else 0.0,
            "ppe_particle_iters_per_s": ppe / wall if wall > 0 else 0.0,
            "peak_resident_bytes": self.peak_bytes,
            "budget_bytes": self.budget,
        }


def requests_from_mix(mix, steps: int) -> List[Request]:
    """Turns cases.serving_mix() output into requests of ``steps`` steps."""
    return [Request(rid=k, arrival=t, case=c, steps=steps) for k, (t, c) in enumerate(mix)]
