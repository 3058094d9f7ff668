"""Runs of the CPU oracle in worker processes, so that long oracle runs
proceed while the GPU side of a parity test executes.  Workers are spawned
(never forked from a process that has touched the GPU)."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

_POOL = None


def pool() -> ProcessPoolExecutor:
    global _POOL
    if _POOL is None:
        n = max(1, min(6, (os.cpu_count() or 2) - 1))
        _POOL = ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"))
    return _POOL


def run_oracle(params: dict, steps: int, f=None, C=None, with_velocity=True):
    """Oracle state after ``steps`` steps: dict of f, C, rho, u, obs, status."""
    import numpy as np  # noqa: F401
    from oracle.observables import observe
    from oracle.solver import Oracle
    o = Oracle(params, f=f, C=C)
    o.step(steps)
    u = o.velocity() if with_velocity else None
    return dict(f=o.f, C=o.C, rho=o.density(), u=u, obs=observe(o.f, o.C, u),
                status=o.status)


def submit(params: dict, steps: int, f=None, C=None):
    return pool().submit(run_oracle, params, steps, f, C)
