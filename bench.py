#!/usr/bin/env python3
"""Benchmark of the SISPH hot path on one MI355X.

A step is one full SISPH time step (binning, predictor, PPE solve,
correction, GTVF, advance) through the C ABI on a seeded synthetic case whose
particles are already resident in HBM.  The headline workload is the 3D dam
break (2,000,000 fluid + 1,343,508 wall particles), the largest
configuration; its value is whole-job PPE throughput: fluid particles x
Jacobi sweeps done in the timed steps, divided by the wall-clock of those
steps (bracketed by device synchronisation).

The JSON line also carries the roofline of the dominant kernel, the Jacobi
sweep (one launch per sweep, or, for a wall-less case that fits on the
device, one persistent launch per solve holding all its sweeps): every
sweep launch is bracketed by its own HIP events on the library's stream
(the wall pressure pass before it left out), and the achieved rate counts
the cached-coefficient method's algorithmic bytes per fluid particle and
sweep (4 B per coefficient over the lattice neighbour count, a neighbour
bitmask over the stencil candidates, 40 B of per-particle data: 420 B in
3D, 128 B in 2D, mixed precision).  The implementation's own stored bytes
and the counter-measured traffic are reported beside it.  A secondary block
measures the 160,000-particle Taylor-Green case, and the CPU oracle (its
OpenMP build, all usable cores) is timed on a bounded sample of the
headline case.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PPE particle-iters/s + HBM GB/s frac; batched vs plain at equal tol; p99 step"
KT_PERIOD = 8   # sweep launches per timed launch in walled cases
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (builder, description)
    "tg400_wendland_mixed": "2D Taylor-Green, periodic unit square, 400x400 lattice (160,000 particles), "
                            "+-1% seeded jitter, Wendland C2 h=1.3dx, Re=100, tol 1e-4, FP32 sums / FP64 "
                            "residual and positions",
    "tg400_wendland_fp64": "same case, all sums FP64",
    "tg50_quintic_fp64": "2D Taylor-Green 50x50, quintic h=dx, Re=100, tol 1e-4, FP64",
    "db2d_dx0.005_mixed": "2D dam break 1x2 column in a 4x4 tank, dx=0.005 (80,000 fluid + 7,218 wall), "
                          "Wendland h=1.3dx, tol 1e-3, mixed",
    "db3d_dx0.01_mixed": "3D dam break 1x1x2 block in a 4x1x4 tank, dx=0.01 (2,000,000 fluid + 1,343,508 wall), "
                         "Wendland h=1.3dx, gravity, free surface, external GTVF, tol 1e-3, mixed",
}


def make_case(name: str):
    from paper_1908_01762_amd import cases
    if name == "tg400_wendland_mixed":
        return cases.taylor_green(400, kernel="wendland", hdx=1.3, precision="mixed", tol=1e-4)
    if name == "tg400_wendland_fp64":
        return cases.taylor_green(400, kernel="wendland", hdx=1.3, precision="fp64", tol=1e-4)
    if name == "tg50_quintic_fp64":
        return cases.taylor_green(50)
    if name == "db2d_dx0.005_mixed":
        return cases.dam_break_2d(dx=0.005, precision="mixed", tol=1e-3)
    if name == "db3d_dx0.01_mixed":
        return cases.dam_break_3d(dx=0.01, precision="mixed", tol=1e-3)
    raise SystemExit(f"unknown workload {name}")


# Algorithmic bytes of one cached-coefficient Jacobi sweep per fluid
# particle: coefficients (4 B mixed, 8 B FP64) over the neighbours of an
# unperturbed lattice without self (2D Wendland h = 1.3 dx: 20, 3D: 80), a
# neighbour bitmask over the stencil candidates (2D 61 bits ~ 8 B, 3D 475 bits
# ~ 60 B), and 40 B of per-particle data (RHS, D_ii, own and new iterate,
# flag, count).
UNIT_BYTES = {(2, "mixed"): 4 * 20 + 8 + 40, (3, "mixed"): 4 * 80 + 60 + 40,
              (2, "fp64"): 8 * 20 + 8 + 40, (3, "fp64"): 8 * 80 + 60 + 40}


def sweep_bytes(case, slots: int, index_bits: int = 32, wall_pairs: int = 0, wall_rows: int = 0,
                list_frac: float = 0.0) -> dict:
    """Bytes the data layout of one Jacobi sweep moves over the whole case.

    Per fluid row: neighbour count (4 B), RHS and D_ii (8 + 8), free-surface
    flag (4), own iterate (8), new iterate (8); mixed adds the FP32 copy of
    the new iterate (4) and reads neighbours' FP32 iterate once (4), FP64
    reads it once (8); the packed mixed sweep reads RHS and D_ii as FP32 and
    count and flag as one word (36 B).  Per stored pair (self slot excluded): neighbour index
    (index_bits: 32, 16 as an offset, 12 as a position in the workgroup's
    LDS copy of the iterate; list_frac of the rows, in workgroups whose copy
    would not fit, read 32-bit list entries instead) and cached coefficient
    (4 mixed, 8 FP64).
    `bytes` is the sweep kernel's.  Cases with walls run the wall pressure
    kernel before every sweep; its bytes are `wall_bytes`: per wall row with
    fluid neighbours (no sweep reads the others, so the kernel skips them)
    the count (4), the hydrostatic term (8) and the new wall pressure (8,
    and its FP32 copy 4 in the mixed mode); per wall pair the cached weight
    and fluid index (8 mixed, 12 FP64).
    """
    nf, nw = case.n_fluid, wall_rows
    pairs = slots - nf
    mixed = case.precision == "mixed"
    row = 4 + 8 + 8 + 4 + 8 + 8 + (4 + 4 if mixed else 8)
    if mixed and index_bits == 12:
        row -= 12   # RHS and D_ii as FP32 (exact: FP32 sums), count and flag in one word
    pair = index_bits / 8 * (1.0 - list_frac) + 4 * list_frac + (4 if mixed else 8)
    total = nf * row + pairs * pair
    wall_row = 4 + 8 + 8 + (4 if mixed else 0)
    wall_pair = 8 if mixed else 12
    wall = nw * wall_row + wall_pairs * wall_pair if nw else 0
    return dict(per_row=row, per_pair=pair, pairs=int(pairs), bytes=int(total), wall_bytes=int(wall),
                wall_rows=int(nw), wall_pairs=int(wall_pairs) if nw else 0,
                per_wall_row=wall_row if nw else 0, per_wall_pair=wall_pair if nw else 0)


def traffic_from_profiles(kernel_src_sha: str, workload: str):
    """HBM traffic per sweep from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"ppe_sweep_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"hbm_bytes_per_sweep:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_src_sha:
        return None
    return float(t.group(1))


def kernel_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("sisph_kernels.hip", "sisph_internal.h"):   # kernels and their launch defaults
        with open(os.path.join(ROOT, "paper_1908_01762_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cpu_baseline(case, budget_s: float) -> dict:
    """The FP64 oracle (its OpenMP build, bitwise equal to the serial one)
    on the first steps of the same case, on every usable host core, for
    about budget_s seconds (at least one step).  The rate counts whole
    steps: the oracle's Jacobi sweeps are only part of them."""
    import oracle
    info = host_info()
    usable = info.get("usable_cpus") or os.cpu_count() or 1
    oracle.set_threads(usable)
    threads = oracle.threads(parallel=True)
    sim = oracle.Sim(case, parallel=True)
    t0 = time.perf_counter()
    iters = steps = 0
    while True:
        out = sim.step()
        iters += out["iters"]
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": case.n_fluid * iters / dt, "unit": "particle-iters/s", "cores": threads, "kind": "oracle",
            "sample": f"first {steps} step(s) of the same case ({iters} Jacobi sweeps, {case.n_fluid} fluid "
                      f"particles), {dt:.1f} s on {threads} host threads; FP64 C oracle, OpenMP build",
            "particle_steps_per_s": case.n_fluid * steps / dt, "host": info}


def host_info() -> dict:
    """The host the oracle ran on: logical CPUs, those this process may use,
    and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def batched_vs_plain(n_cases: int, steps: int, seed: int) -> dict:
    """The same uneven cases (serving mix: Taylor-Green or 2D dam break, N
    log-uniform in 2.5k-160k, their own tolerances) stepped three ways from
    the same initial state for the same number of steps: one case at a time
    with its own launches in the plain FP32 mode (the baseline: every sum,
    the residual and the stopping test in FP32) and in the mixed mode, and
    all together as one batch in the mixed mode (FP32 neighbour sums, FP64
    residual and positions).  The tolerance is the same for all three;
    mixed plain and batched take identical sweeps."""
    import torch
    from paper_1908_01762_amd import cases, sisph
    mix = [c for _, c in cases.serving_mix(n_cases=n_cases, seed=seed)]
    nf = sum(c.n_fluid for c in mix)

    def per_case(precision):
        ctxs = [sisph.Context(c.replace(precision=precision)) for c in mix]
        for ctx in ctxs:          # one warm step each (first-step p_ref, caches)
            ctx.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for ctx in ctxs:
            its += sum(s["iters"] * ctx.case.n_fluid for s in ctx.step(steps))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        for ctx in ctxs:
            ctx.close()
        return el, its

    plain32_s, it32 = per_case("fp32")
    plain_s, it_plain = per_case("mixed")
    ctxs = [sisph.Context(c) for c in mix]
    b = sisph.Batch(len(ctxs))
    for ctx in ctxs:
        b.attach(ctx)
    b.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_batch = 0
    for _ in range(steps):
        it_batch += sum(s["iters"] * c.case.n_fluid for s, c in zip(b.step(), ctxs))
    torch.cuda.synchronize()
    batched = time.perf_counter() - t0
    b.close()
    for ctx in ctxs:
        ctx.close()
    return {"cases": len(mix), "fluid_particles": nf, "steps": steps,
            "plain_fp32_s": plain32_s, "plain_mixed_s": plain_s, "batched_mixed_s": batched,
            "speedup_vs_plain_fp32": plain32_s / batched, "speedup_vs_plain_mixed": plain_s / batched,
            "plain_fp32_ppe_particle_iters_per_s": it32 / plain32_s,
            "plain_mixed_ppe_particle_iters_per_s": it_plain / plain_s,
            "batched_ppe_particle_iters_per_s": it_batch / batched,
            "plain_fp32_particle_steps_per_s": nf * steps / plain32_s,
            "batched_particle_steps_per_s": nf * steps / batched,
            "same_sweep_counts_mixed": it_plain == it_batch,
            "workload": "serving mix (seed %d): Taylor-Green / 2D dam break, N log-uniform 2.5k-160k, "
                        "tol 1e-4 (TG) / 1e-3 (dam break)" % seed}


def copy_reference(sizes_mib=(32, 1024), reps: int = 20) -> list:
    """Device-to-device copies (torch, i.e. the runtime's copy kernel) of the
    given sizes timed with events: the bandwidth a plain streaming kernel
    reaches, read + write counted; and a plain read of the same buffer."""
    import torch
    from paper_1908_01762_amd import sisph
    out = []
    for mib in sizes_mib:
        n = mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        # a plain read of the same buffer (the library's read probe): the
        # rate a kernel that only reads, as the sweep nearly does, can reach
        grid = 2048
        out_buf = torch.empty(grid * 256, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        rus = sisph.read_rate(src.data_ptr(), n * 4, out_buf.data_ptr(), grid, reps)
        out.append({"mib": mib, "us": round(us, 3), "GBps": round(2 * n * 4 / (us * 1e-6) / 1e9, 1),
                    "read_us": round(rus, 3), "read_GBps": round(n * 4 / (rus * 1e-6) / 1e9, 1)})
        del src, dst, out_buf
    return out


def solver_compare(dx: float, steps: int, tols=(1e-2, 1e-3, 1e-4)) -> dict:
    """Jacobi (the paper's scheme) against BiCGStab on the same cached
    operator at equal tolerance: 2D dam break (free surface, so the system is
    non-singular), mixed precision, the same initial state and step count
    for both.  Operator applications: one per Jacobi sweep, two per BiCGStab
    iteration plus one for the initial residual."""
    import torch
    from paper_1908_01762_amd import cases, sisph
    out = {"workload": f"2D dam break dx={dx} (mixed), {steps} steps after one warm step", "rows": []}
    for tol in tols:
        for solver in ("jacobi", "bicgstab"):
            case = cases.dam_break_2d(dx=dx, precision="mixed", tol=tol).replace(solver=solver, max_iter=20000)
            ctx = sisph.Context(case)
            ctx.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.step(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            its = [s["iters"] for s in st]
            ops = sum(its) if solver == "jacobi" else sum(2 * k + 1 for k in its)
            out["rows"].append({"tol": tol, "solver": solver, "fluid_particles": case.n_fluid,
                                "mean_iters": sum(its) / len(its), "operator_applications": ops,
                                "ms_per_step": el * 1e3 / steps,
                                "all_converged": all(s["converged"] for s in st)})
            ctx.close()
    return out


def serving(n_requests: int, steps: int, rate_hz: float, budget_gb: float, seed: int) -> dict:
    """Continuous batching: Poisson arrivals, admission by workspace bytes."""
    from paper_1908_01762_amd import cases
    from paper_1908_01762_amd.serve import GpuBackend, Server, requests_from_mix
    reqs = requests_from_mix(cases.serving_mix(n_cases=n_requests, seed=seed, rate_hz=rate_hz), steps)
    backend = GpuBackend(max_slots=n_requests)
    srv = Server(backend, budget_bytes=int(budget_gb * 1e9), max_slots=n_requests, keep_results=False)
    rep = srv.run(reqs)
    backend.close()
    rep.update(requests_per_s_offered=rate_hz, steps_per_request=steps)
    return rep


def measure(workload: str, steps: int, warmup: int, launch: str, autotune: bool, persistent: bool = True,
            variant: int = -1) -> dict:
    """Steps one case: warmup steps, the autotuner, then `steps` timed steps
    with every sweep kernel launch timed by its own HIP events."""
    import torch
    from paper_1908_01762_amd import sisph
    case = make_case(workload)
    ctx = sisph.Context(case, device="cuda:0")
    if launch == "graphs":
        ctx.use_graphs(True)
    if not persistent:
        ctx.use_persistent(False)
    print(f"[bench] workload {workload}: {case.n_fluid} fluid + {case.n_wall} wall particles, "
          f"workspace {ctx.nbytes / 1e6:.1f} MB", file=sys.stderr, flush=True)
    warm = ctx.step(warmup) if warmup else []
    tuned = None
    if variant >= 0:
        ctx.variant = variant
        tuned = {"variant": variant, "forced": True}
    elif warmup and autotune:
        # the project's autotuner picks the sweep launch variant on the live
        # state (outside the timed region; variants change speed only)
        best, us = ctx.autotune(20)
        tuned = {"variant": best, "us_per_variant": [round(t, 3) for t in us]}
        print(f"[bench] autotuned sweep variant {best}", file=sys.stderr, flush=True)
    # every sweep launch of a walled case timed by its own event pair would
    # slow the run it measures (a few us per pair): there every KT_PERIOD-th
    # launch of a solve is timed, and the per-launch average stands for all
    period = KT_PERIOD if case.n_wall else 1
    ctx.set_kernel_timing(period)
    torch.cuda.synchronize()
    ctx.sweep_counters(reset=True)
    t0 = time.perf_counter()
    stats = ctx.step(steps) if steps > 0 else []
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {workload}: timed {steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # per-step sweep counts of this process's solves, warmup first (the
    # profile summaries turn per-launch counters into per-sweep figures)
    counts = [s["iters"] for s in warm] + [s["iters"] for s in stats]
    print(f"[bench] solve sweep counts: {counts}", file=sys.stderr, flush=True)
    iters = sum(s["iters"] for s in stats)
    value = case.n_fluid * iters / elapsed if elapsed > 0 else 0.0
    cnt = ctx.sweep_counters()
    kt = ctx.kernel_timing()
    pinfo = ctx.persistent_info()
    fallbacks = ctx.persistent_fallbacks()   # since the reset: the timed steps only
    wall_rows = ctx.rows_with_neighbours(1, 1) if case.n_wall else 0
    nblk = -(-case.n_fluid // 256)
    list_blocks = stats[-1]["list_blocks"] if stats else 0
    sb = sweep_bytes(case, ctx.pair_count(1, 0), index_bits=stats[-1]["index_bits"] if stats else 32,
                     wall_pairs=ctx.pair_count(1, 1) if case.n_wall else 0, wall_rows=wall_rows,
                     list_frac=list_blocks / nblk)
    unit = UNIT_BYTES[(case.dim, case.precision)]
    # the dominant kernel: the sweep, one launch per sweep, or one persistent
    # launch per solve holding its sweeps; both are timed by their own events
    n_persistent = kt["persistent"]
    # every launch when each is timed; else (walled cases: per-sweep
    # launches only) the sweep counter's launches
    all_launches = kt["launches"] if period == 1 else cnt["launches"]
    n_perlaunch = all_launches - n_persistent
    if n_persistent and n_perlaunch:
        mode = "mixed"
    elif n_persistent:
        mode = "persistent"
    else:
        mode = "per-sweep launches"
    timed = kt["launches"]
    avg_launch_s = kt["ms"] / 1e3 / max(timed, 1)
    # the sampled average over every launch (exact when period is 1)
    kernel_s = kt["ms"] / 1e3 if period == 1 else avg_launch_s * all_launches
    launches = all_launches
    eff = cnt["effective"]
    alg_per_sweep = unit * case.n_fluid
    achieved = alg_per_sweep * eff / kernel_s / 1e9 if kernel_s > 0 else 0.0
    layout_rate = sb["bytes"] * eff / kernel_s / 1e9 if kernel_s > 0 else 0.0
    traffic = traffic_from_profiles(kernel_sha(), workload)
    kernel = {"persistent": "k_ppe_persistent (one launch per solve)", "per-sweep launches": "Sweep",
              "mixed": "k_ppe_persistent + Sweep"}[mode]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic * eff / max(launches, 1)) if traffic is not None else None,
                # the counter-measured bytes (the committed summary's, per
                # sweep) over the same kernel time: the HBM-side rate
                "traffic_GBps": round(traffic * eff / kernel_s / 1e9, 1) if traffic is not None and kernel_s > 0
                else None,
                "traffic_frac": round(traffic * eff / kernel_s / 1e9 / HBM_PEAK_GBS, 4)
                if traffic is not None and kernel_s > 0 else None,
                "kernel": kernel, "mode": mode,
                "algorithmic_bytes_per_particle_iter": unit,
                "algorithmic_bytes_per_sweep": alg_per_sweep,
                "algorithmic_bytes_per_launch": int(round(alg_per_sweep * eff / max(launches, 1))),
                "avg_launch_us": round(avg_launch_s * 1e6, 3), "launches": launches,
                "timed_launches": timed, "timing_period": period,
                "persistent_launches": n_persistent, "per_sweep_launches": n_perlaunch,
                "effective_sweeps": eff,
                "avg_us_per_effective_sweep": round(kernel_s * 1e6 / max(eff, 1), 3),
                "persistent_fallbacks": fallbacks,
                "note": ("the cached-coefficient method's bytes over the sweep time; the persistent solve keeps "
                         "its coefficients in registers and is bound by its grid barrier, not by HBM")
                if n_persistent else ("the cached-coefficient method's bytes over the sweep kernel's time; "
                                      "the kernel streams its coefficients and codes from HBM"),
                "layout": {"bytes_per_sweep": sb["bytes"], "bytes_per_row": sb["per_row"],
                           "bytes_per_pair": round(sb["per_pair"], 4), "pairs": sb["pairs"],
                           "index_bits": stats[-1]["index_bits"] if stats else 32, "list_blocks": list_blocks,
                           "achieved_GBps": round(layout_rate, 1),
                           "traffic_per_sweep": round(traffic) if traffic is not None else None}}
    if case.n_wall:
        # the wall pressure pass runs before every sweep, outside the timed
        # sweep kernel: its share of the chunk time (with the launch gaps)
        # and its own bytes
        roofline["wall_pass"] = {"rows": sb["wall_rows"], "pairs": sb["wall_pairs"],
                                 "bytes_per_row": sb["per_wall_row"], "bytes_per_pair": sb["per_wall_pair"],
                                 "bytes_per_sweep": sb["wall_bytes"],
                                 "us_per_sweep": round((cnt["sweep_ms"] - kernel_s * 1e3) * 1e3 /
                                                       max(cnt["launches"], 1), 3)}
    out = {
        "value": value,
        "ms_per_step": elapsed * 1e3 / max(steps, 1),
        "dtype": "f32+f64" if case.precision == "mixed" else "f64",
        "config": {"workload": workload, "description": WORKLOADS[workload],
                   "fluid_particles": case.n_fluid, "wall_particles": case.n_wall,
                   "launch": launch, "parallelism": "single GPU"},
        "mean_ppe_iters": iters / max(len(stats), 1),
        "solves_at_max_iter": sum(1 for s in stats if s["iters"] >= case.max_iter),
        "particle_steps_per_s": case.n_fluid * steps / elapsed if elapsed > 0 else 0.0,
        "sweep_time_frac": cnt["sweep_ms"] / 1e3 / elapsed if elapsed > 0 else 0.0,
        "roofline": roofline,
        "sweep_variant": tuned if tuned is not None else {"variant": ctx.variant},
        # external-flow GTVF: did the last timed step's sub-steps walk the
        # short lists (1), the full lists for some sub-step (2), or has the
        # case none (0)
        "gtvf_short_lists_last_step": ctx.debug_gtvf_short(),
    }
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="db3d_dx0.01_mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary", default="tg400_wendland_mixed", choices=sorted(WORKLOADS) + ["none"],
                    help="a second workload measured the same way and reported under 'secondary'")
    ap.add_argument("--secondary-steps", type=int, default=195)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-compare", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--batch-cases", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gb", type=float, default=1.0)
    ap.add_argument("--no-solver-compare", action="store_true")
    ap.add_argument("--compare-dx", type=float, default=0.01)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default sweep variant instead of autotuning it after the warmup")
    ap.add_argument("--variant", type=int, default=-1,
                    help="launch the main workload's sweeps with this variant instead of autotuning "
                         "(counter runs that must replay the benchmark's kernel)")
    ap.add_argument("--launch", choices=("eager", "graphs"), default="eager",
                    help="launch the fixed parts of each step one kernel at a time, or replay them "
                         "from HIP graphs")
    ap.add_argument("--no-persistent", action="store_true",
                    help="solve wall-less cases with per-sweep launches instead of one persistent launch")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a counter calibration "
                         "reference for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(sharding one case over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_01762_amd import sisph

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    sisph.lib()
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written",
              file=sys.stderr, flush=True)
        del src, dst
    primary = measure(args.workload, args.steps, args.warmup, args.launch, not args.no_autotune,
                      not args.no_persistent, args.variant)
    line = {
        "metric": METRIC,
        "value": primary.pop("value"),
        "unit": "particle-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": primary.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": primary.pop("dtype"),
        "data": "synthetic",
        "config": primary.pop("config"),
    }
    line.update(primary)
    if args.secondary != "none" and args.secondary != args.workload:
        print(f"[bench] secondary workload {args.secondary}", file=sys.stderr, flush=True)
        line["secondary"] = measure(args.secondary, args.secondary_steps, args.warmup, args.launch,
                                    not args.no_autotune, not args.no_persistent)
    if not args.no_batch_compare:
        print("[bench] batched vs plain", file=sys.stderr, flush=True)
        line["batched_vs_plain"] = batched_vs_plain(args.batch_cases, args.batch_steps, seed=0)
    line["copy_reference"] = copy_reference()
    big = [c for c in line["copy_reference"] if c["mib"] == 1024]
    if big and big[0]["read_GBps"] > 0:
        # context for frac: the rate a plain read of 1 GiB reaches on this device
        rf = line["roofline"]
        rf["read_probe_GBps"] = big[0]["read_GBps"]
        rf["frac_of_read_probe"] = round(rf["achieved"] / big[0]["read_GBps"], 4)
    if not args.no_solver_compare:
        print("[bench] Jacobi vs BiCGStab", file=sys.stderr, flush=True)
        line["solver_compare"] = solver_compare(args.compare_dx, args.batch_steps)
    if not args.no_serving:
        print("[bench] serving", file=sys.stderr, flush=True)
        line["serving"] = serving(args.serve_requests, args.serve_steps, args.serve_rate,
                                  args.serve_budget_gb, seed=1)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(make_case(args.workload), args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
