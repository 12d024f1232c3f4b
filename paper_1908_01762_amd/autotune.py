"""Autotuner for the Jacobi-sweep launch variant, with a JSON cache.

The library times its sweep variants on a case's live state
(``sisph_autotune``); this driver keys the winner by (dimension, kernel,
precision, size bucket = round(log2 N_fluid)) and stores it, so later cases
of the same kind reuse the choice without timing.  Variants change the
speed only, never the result.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sisph_autotune.json")


def key(case) -> str:
    bucket = int(round(math.log2(max(case.n_fluid, 1))))
    return f"d{case.dim}-{case.kernel}-{case.precision}-n2^{bucket}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cached(ctx, cache_path: Optional[str] = None) -> bool:
    """Sets the cached variant for this kind of case; False if none."""
    data = _load(cache_path or DEFAULT_CACHE)
    hit = data.get(key(ctx.case))
    if hit is None:
        return False
    ctx.variant = int(hit["variant"])
    return True


def tune(ctx, cache_path: Optional[str] = None, reps: int = 20, force: bool = False) -> dict:
    """Uses the cache, or times the variants on ctx (after one completed step)
    and records the winner."""
    path = cache_path or DEFAULT_CACHE
    k = key(ctx.case)
    data = _load(path)
    if not force and k in data:
        ctx.variant = int(data[k]["variant"])
        return data[k]
    best, us = ctx.autotune(reps)
    ctx.variant = best
    data[k] ={"variant": best, "us": [round(t, 3) for t in us], "n_fluid": ctx.case.n_fluid}
    _store(path, data)
    return data[k]
