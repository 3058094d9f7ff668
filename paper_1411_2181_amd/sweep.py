"""Batched droplet runs and critical-capillary-number searches (host driver).

The paper locates Ca_cr for each (De, lambda, 2R/W) by finding the largest
wall speed at which the droplet is stable and the smallest at which it
breaks (Section 3, set-up paragraph).  Here each search is a bisection in Ca
whose runs are advanced together in one batched context (every round of
every query triple in one launch sequence); break-up is a droplet split into
two or more pieces of at least 1 % of its volume (6-connected components).

Lattice mapping (physics.lattice_params): Shan-Chen G = 0.75, matrix solvent
tau = 1.5 (the top of the calibrated window), U_w <= 0.19; the box is (16R) x (3R) x (2R/c): long enough in
the flow direction that an elongated droplet breaks instead of joining its
periodic image.  The reachable Ca range depends on (c, lambda) through the
wall-speed cap and is reported with every search.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbmve, physics

TAU_MATRIX = 1.5
U_MAX = 0.19
BOX_X = 16.0


@dataclass
class RunSpec:
    R: float
    c: float            # confinement 2R/W
    Ca: float
    De: float = 0.0
    lam: float = 1.0
    L2: float = 100.0
    fraction: float = 0.4
    phase: str = "DV"

    def inputs(self):
        """Surrogate inputs: (Ca, De, lambda, 2R/W, L^2, polymer fraction)."""
        return [self.Ca, self.De, self.lam, self.c, self.L2, self.fraction]


@dataclass
class RunResult:
    spec: RunSpec
    params: dict
    info: dict
    broken: bool = False
    step_break: int = -1
    steps: int = 0
    D: float = float("nan")
    theta: float = float("nan")
    Lp_max: float = 0.0
    status: int = 0
    history: list = field(default_factory=list)


def box(R: float, c: float):
    return int(round(BOX_X * R)), int(round(3.0 * R)), int(round(2.0 * R / c))


def ca_max(R: float, c: float, lam: float, De: float = 0.0, fraction: float = 0.4,
           phase: str = "DV") -> float:
    """Largest Ca reachable at U_w = U_MAX for this geometry and viscosity ratio."""
    nx, ny, nz = box(R, c)
    eta_B = physics.eta_of_tau(TAU_MATRIX)
    eta_M = eta_B if phase in ("DV", "N") else eta_B / (1.0 - fraction)
    eta_d = lam * eta_M
    eta_A = eta_d * (1.0 - fraction) if (phase == "DV" and De > 0) else eta_d
    if phase == "MV":
        eta_A = lam * eta_M
    tau_A = physics.tau_of_eta(eta_A)
    sig = physics.sigma_for(tau_A, TAU_MATRIX)
    return U_MAX * 2.0 * eta_M * R / (sig * nz)


def lattice(spec: RunSpec):
    nx, ny, nz = box(spec.R, spec.c)
    phase = spec.phase if spec.De > 0 else "N"
    p, info = physics.lattice_params(nx, ny, nz, spec.R, spec.Ca, spec.De, spec.lam, phase=phase,
                                     L2=spec.L2, fraction=spec.fraction, tau_matrix=TAU_MATRIX,
                                     u_max=U_MAX * (1 + 1e-9))
    return p, info


def simulate(specs, precision: str = "fp32", t_end: int | None = None, every: int = 1000,
             min_steps: int = 4000, max_steps: int = 40000, device="cuda:0", launch=None):
    """Advance every run (one batch) to its end time, checking for break-up
    every ``every`` steps; a broken run is stopped (masked) at once.  Steady
    D and orientation are averaged over the last three checks of unbroken
    runs.  Returns (results, seconds)."""
    results, runs = [], []
    for sp in specs:
        p, info = lattice(sp)
        results.append(RunResult(sp, p, info))
        runs.append(p)
    ends = []
    for r in results:
        te = t_end if t_end is not None else physics.run_length(r.info["tau_em"], lo=min_steps,
                                                                hi=max_steps)
        ends.append(int(te))
    import torch
    t0 = time.perf_counter()
    b = lbmve.Batch(runs, precision, device=device)
    if launch:
        b.set_launch(**launch)
    remaining = list(ends)
    while max(remaining) > 0:
        chunk = [min(every, r) for r in remaining]
        b.step(chunk)
        obs = b.observe(components=True)
        for k, (r, o) in enumerate(zip(results, obs)):
            if chunk[k] == 0:
                continue
            remaining[k] -= chunk[k]
            r.steps = o["step"]
            r.status = o["status"]
            r.history.append((o["step"], o["D"], o["theta_deg"], o["Lp"], o["n_components"]))
            r.Lp_max = max(r.Lp_max, o["Lp"])
            if o["status"] != 0:
                remaining[k] = 0
            elif o["n_components"] >= 2:
                r.broken = True
                r.step_break = o["step"]
                remaining[k] = 0
    torch.cuda.synchronize()
    b.close()
    for r in results:
        tail = [h for h in r.history[-3:]]
        if not r.broken and tail:
            r.D = float(np.mean([h[1] for h in tail]))
            r.theta = float(np.mean([h[2] for h in tail]))
    return results, time.perf_counter() - t0


@dataclass
class Search:
    De: float
    lam: float
    c: float
    R: float
    lo: float
    hi: float
    lo_ok: bool = False      # lo verified stable
    hi_ok: bool = False      # hi verified broken
    runs: int = 0
    done: bool = False
    outside: str = ""        # "below" / "above" when Ca_cr is outside the range

    @property
    def ca_cr(self):
        return 0.5 * (self.lo + self.hi)


def bisect(searches, tol: float = 0.02, precision: str = "fp32", verify_ends: bool = True,
           max_rounds: int = 12, **sim_kw):
    """Bisection in Ca for every search at once.  If ``verify_ends``, the
    first round simulates both bracket ends (a proposed bracket must be
    confirmed: lo stable, hi broken); a failed end widens the bracket toward
    the hard limits [0.02, Ca_max].  Returns (searches, seconds, rounds)."""
    total = 0.0
    rounds = 0
    for s in searches:
        s.hard_lo, s.hard_hi = 0.02, ca_max(s.R, s.c, s.lam, s.De)
        s.hi = min(s.hi, s.hard_hi)
        s.lo = max(s.lo, s.hard_lo)
    while rounds < max_rounds:
        todo, specs = [], []
        for s in searches:
            if s.done:
                continue
            if verify_ends and not s.lo_ok:
                todo.append((s, "lo"))
                specs.append(RunSpec(s.R, s.c, s.lo, s.De, s.lam))
            if verify_ends and not s.hi_ok:
                todo.append((s, "hi"))
                specs.append(RunSpec(s.R, s.c, s.hi, s.De, s.lam))
            if (s.lo_ok and s.hi_ok) or not verify_ends:
                if s.hi - s.lo <= tol:
                    s.done = True
                    continue
                todo.append((s, "mid"))
                specs.append(RunSpec(s.R, s.c, 0.5 * (s.lo + s.hi), s.De, s.lam))
        if not todo:
            break
        res, sec = simulate(specs, precision, **sim_kw)
        total += sec
        rounds += 1
        for (s, what), r in zip(todo, res):
            s.runs += 1
            if what == "lo":
                if not r.broken:
                    s.lo_ok = True
                elif s.lo <= s.hard_lo + 1e-12:
                    s.done, s.outside = True, "below"
                else:
                    # the proposed lower end already breaks: fall back to the
                    # full lower range
                    s.hi, s.hi_ok = s.lo, True
                    s.lo, s.lo_ok = s.hard_lo, False
            elif what == "hi":
                if r.broken:
                    s.hi_ok = True
                elif s.hi >= s.hard_hi - 1e-12:
                    s.done, s.outside = True, "above"
                else:
                    s.lo, s.lo_ok = s.hi, True
                    s.hi, s.hi_ok = s.hard_hi, False
            else:
                mid = 0.5 * (s.lo + s.hi)
                if r.broken:
                    s.hi = mid
                else:
                    s.lo = mid
        for s in searches:
            if not s.done and s.lo_ok and s.hi_ok and s.hi - s.lo <= tol:
                s.done = True
    return searches, total, rounds
