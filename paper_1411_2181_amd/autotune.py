"""Launch-shape autotuner for the step kernels.

Times a few steps of a solver or batch for each candidate tile shape
(bx, by, bz, persistent) with the library's event-timed steps and keeps the
fastest.  Results are cached per (device, precision, size bucket, polymer)
in a JSON file so repeated runs reuse them.  Every shape gives bit-identical
fields, so tuning never changes results, only speed.
"""
from __future__ import annotations

import json
import math
import os
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "autotune_cache.json")

SHAPES = [(32, 8), (16, 16), (16, 8), (8, 16)]
# the FP64 rings of the 512-thread tiles exceed the LDS
SHAPES_FP64 = [(16, 8), (8, 16)]
BZ = [16, 32, 64, 128]      # planes per tile; 0 (also tried): whole columns
PERSISTENT = [1024, 2048]


def candidates(nz_max: int, precision: str = "fp32"):
    shapes = SHAPES_FP64 if precision == "fp64" else SHAPES
    out = []
    for bx, by in shapes:
        for bz in BZ + [0]:
            if bz <= max(8, nz_max) and not (bz == 0 and nz_max in BZ):
                out.append(dict(bx=bx, by=by, bz=bz, persistent=0))
    return out


def _key(batch) -> str:
    import torch
    name = torch.cuda.get_device_name(batch.device)
    nodes = sum(d["nx"] * d["ny"] * d["nz"] for d in batch.dicts)
    bucket = int(round(math.log2(max(nodes, 1))))
    visc = any(max(d["eta_P"]) > 0 for d in batch.dicts)
    return f"{name}|{batch.precision}|2^{bucket}|runs{batch.nruns}|visc{int(visc)}"


def _load():
    if os.path.exists(CACHE):
        try:
            with open(CACHE) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def tune(batch, steps: int = 4, cands=None, use_cache: bool = True, save: bool = True,
         persistent: bool = True) -> dict:
    """Pick the fastest launch shape for ``batch`` (an lbmve.Batch/Solver),
    apply it and return {"launch": ..., "ms_per_step": ..., "table": [...]}.

    Tuning advances the runs by (len(cands) + len(PERSISTENT) + 1) * steps
    steps; callers that need a pristine state tune on a scratch copy."""
    key = _key(batch)
    cache = _load()
    if use_cache and key in cache:
        batch.set_launch(**cache[key]["launch"])
        return dict(cache[key], cached=True)
    nz_max = max(d["nz"] for d in batch.dicts)
    cands = cands or candidates(nz_max, batch.precision)
    table = []
    batch.step_profiled(steps)          # warm-up: graph-free, first-touch
    for c in cands:
        batch.set_launch(**c)
        ms = batch.step_profiled(steps) / steps
        table.append(dict(launch=c, ms_per_step=ms))
    best = min(table, key=lambda r: r["ms_per_step"])
    # persistent grids of the best shape (a few workgroups per CU looping over
    # the tile table)
    for pers in (PERSISTENT if persistent else []):
        c = dict(best["launch"], persistent=pers)
        batch.set_launch(**c)
        ms = batch.step_profiled(steps) / steps
        table.append(dict(launch=c, ms_per_step=ms))
    best = min(table, key=lambda r: r["ms_per_step"])
    batch.set_launch(**best["launch"])
    res = dict(launch=best["launch"], ms_per_step=best["ms_per_step"], table=table,
               when=time.strftime("%Y-%m-%d %H:%M:%S"))
    if save:
        cache[key] = res
        try:
            with open(CACHE, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return dict(res, cached=False)
