"""Writes tg400_decay_series.json: the FP64 oracle's maximum-velocity decay
over 200 steps of the 160,000-particle Taylor-Green case (400 x 400 lattice,
+-1% jitter seed 0, Wendland C2 h = 1.3 dx, Re = 100, eps = 1e-4, the R24
projection of the periodic PPE).

Calls only the oracle (its OpenMP build, bitwise equal to the serial one)
and the seeded case generator; nothing from the HIP path.  Run from the
repository root: python tests/golden/make_tg400_series.py
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1908_01762_amd import cases  # noqa: E402

STEPS = 200


def main():
    case = cases.taylor_green(400, kernel="wendland", hdx=1.3, tol=1e-4, seed=0)
    sim = oracle.Sim(case, parallel=True)
    u0 = float(np.linalg.norm(case.u, axis=1).max())
    t, ratio, iters = [], [], []
    t0 = time.time()
    for k in range(STEPS):
        out = sim.step()
        t.append(sim.t)
        ratio.append(float(np.linalg.norm(sim.u, axis=1).max()) / u0)
        iters.append(int(out["iters"]))
        if k % 20 == 19:
            print(f"step {k + 1}: |u|max ratio {ratio[-1]:.9f}, {time.time() - t0:.0f} s", flush=True)
    doc = {
        "what": "|u|max(t) / |u|max(0) of the FP64 oracle, 160k-particle Taylor-Green",
        "case": {"lattice": 400, "kernel": "wendland", "hdx": 1.3, "re": 100.0, "jitter": 0.01, "seed": 0,
                 "tol": 1e-4, "null_space": case.null_space, "dt": case.dt, "steps": STEPS},
        "exact_end": math.exp(-8.0 * math.pi ** 2 / 100.0 * t[-1]),
        "t": t, "umax_ratio": ratio, "iters": iters,
    }
    with open(os.path.join(HERE, "tg400_decay_series.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
