"""Solver-variant studies on the same kernels (GPU).

* tolerance_sweep: the Taylor-Green vortex on a 100x100 lattice with the PPE
  tolerance varied over the paper's range (section 4.1, "change in
  tolerance"): mean Jacobi sweeps per step and the decay of |u|max against
  exp(-8 pi^2 t / Re).
* eisph_vs_sisph: one forced Jacobi sweep per step (EISPH, the explicit
  scheme the paper compares against) versus iterating to the tolerance, at
  a high Reynolds number (section 4.1, "comparison with EISPH").

Both return plain dicts; all compute runs through libsisph.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from . import cases

PAPER_TOLERANCES = (0.1, 0.05, 1e-2, 5e-3, 1e-3, 5e-4)


def _decay_run(case, steps: int) -> Dict[str, float]:
    from . import sisph
    ctx = sisph.Context(case)
    u0 = float(np.linalg.norm(case.u, axis=1).max())
    re = case.meta["re"]
    b = -8.0 * math.pi ** 2 / re
    iters: List[int] = []
    worst = 0.0
    t = 0.0
    for _ in range(steps):
        iters.append(ctx.step(1)[0]["iters"])
        t += case.dt
        st = ctx.read_state()
        umax = float(np.linalg.norm(st["u"], axis=1).max())
        if not np.isfinite(umax):
            worst = float("inf")
            break
        worst = max(worst, abs(umax / u0 - math.exp(b * t)))
    ctx.close()
    return {"mean_sweeps": float(np.mean(iters)), "max_sweeps": int(max(iters)),
            "decay_error_max": worst, "t_end": t}


def tolerance_sweep(n: int = 100, steps: int = 100, tolerances: Sequence[float] = PAPER_TOLERANCES,
                    re: float = 100.0, precision: str = "mixed") -> List[Dict[str, float]]:
    out = []
    for tol in tolerances:
        case = cases.taylor_green(n, tol=tol, re=re, precision=precision)
        r = _decay_run(case, steps)
        r["tol"] = tol
        out.append(r)
    return out


def eisph_vs_sisph(n: int = 100, steps: int = 100, re: float = 10000.0, tol: float = 1e-2,
                   precision: str = "mixed") -> Dict[str, Dict[str, float]]:
    sisph_case = cases.taylor_green(n, tol=tol, re=re, precision=precision)
    eisph_case = sisph_case.replace(forced_iters=1, min_iter=1)
    return {"sisph": _decay_run(sisph_case, steps), "eisph": _decay_run(eisph_case, steps)}
