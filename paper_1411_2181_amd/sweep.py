"""Batched droplet runs and critical-capillary-number searches (host driver).

The paper locates Ca_cr for each (De, lambda, 2R/W) by finding the largest
wall speed at which the droplet is stable and the smallest at which it
breaks (Section 3, set-up paragraph).  Here each search is a bisection in Ca
whose runs are advanced together in one batched context (every query's runs
of a round in one launch sequence); break-up is a droplet split into two or
more pieces of at least 1 % of its volume (6-connected components).

Lattice mapping (physics.lattice_params): Shan-Chen G = 0.75, matrix solvent
tau = 1.5 (the top of the calibrated window), U_w <= 0.19; the box is
(16R) x (3R) x (2R/c): long enough in the flow direction that an elongated
droplet breaks instead of joining its periodic image.  Ca_max, the Ca at the
wall-speed cap, is eta_M c U_max / sigma: it does not depend on R, and it
bounds every search window.
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
    tau_matrix: float = 0.0    # matrix solvent relaxation time; 0: TAU_MATRIX

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
    pieces: list = field(default_factory=list)   # node counts of the pieces at break-up
    history: list = field(default_factory=list)
    extended: bool = False   # ran past its end time because it was still elongating


def still_elongating(history, window: int = 4000) -> bool:
    """True when the droplet's length L_p at the last check exceeds its length
    ``window`` steps earlier (the latest check at or before that step).  A
    droplet that stays whole relaxes or holds its length; one that is still
    stretching at the end of a run may yet break."""
    if not history:
        return False
    last_step, last_lp = history[-1][0], history[-1][3]
    earlier = [h for h in history if h[0] <= last_step - window]
    return bool(earlier) and last_lp > earlier[-1][3]


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
                                     L2=spec.L2, fraction=spec.fraction,
                                     tau_matrix=spec.tau_matrix or TAU_MATRIX,
                                     u_max=U_MAX * (1 + 1e-9))
    return p, info


def simulate(specs, precision: str = "fp32", t_end: int | None = None, every: int = 1000,
             min_steps: int = 4000, max_steps: int = 40000, device="cuda:0", launch=None,
             progress=None, extend_to: int = 0, grow_window: int = 4000, prepared=None):
    """Advance every run (one batch) to its end time, checking for break-up
    every ``every`` steps; a broken run is stopped (masked) at once.  With
    ``extend_to`` > 0, a run still whole at its end time whose droplet is
    still elongating (still_elongating over ``grow_window`` steps) goes on,
    check by check, until it breaks, stops elongating or reaches
    ``extend_to`` steps.  Steady D and orientation are averaged over the last
    three checks of unbroken runs; ``progress`` (a callable) receives a line
    after every check.  ``prepared`` (a list of (params, info), one per
    spec) replaces the study window's mapping of the specs to lattice
    parameters.  Returns (results, seconds)."""
    results, runs = [], []
    for k, sp in enumerate(specs):
        p, info = prepared[k] if prepared is not None else lattice(sp)
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
            # (step, D, theta, L_p, pieces, nodes of the four largest pieces)
            r.history.append((o["step"], o["D"], o["theta_deg"], o["Lp"], o["n_components"],
                              sum(o["piece_nodes"])))
            r.Lp_max = max(r.Lp_max, o["Lp"])
            if o["status"] != 0:
                remaining[k] = 0
            elif o["n_components"] >= 2:
                r.broken = True
                r.step_break = o["step"]
                r.pieces = [v for v in o["piece_nodes"] if v > 0]
                remaining[k] = 0
            elif (remaining[k] == 0 and extend_to > r.steps
                  and still_elongating(r.history, grow_window)):
                r.extended = True
                remaining[k] = min(every, extend_to - r.steps)
        if progress:
            progress(f"  step {max(r.steps for r in results)}: "
                     f"{sum(1 for v in remaining if v > 0)} running, "
                     f"{sum(r.broken for r in results)} broken, {time.perf_counter() - t0:.1f} s")
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
    """One Ca_cr search: the bracket [lo, hi] (lo stable, hi broken once
    verified) inside the hard window [hard_lo, hard_hi]."""
    De: float
    lam: float
    c: float
    R: float
    lo: float
    hi: float
    hard_lo: float = 0.0
    hard_hi: float = 0.0
    L2: float = 100.0
    fraction: float = 0.4
    lo_ok: bool = False      # lo verified (or assumed) stable
    lo_assumed: bool = False # lo is the window's bottom, taken as stable without a run
    hi_ok: bool = False      # hi verified broken
    speculate: bool = True   # run the midpoint alongside unverified ends
    runs: int = 0
    rounds: int = 0
    updates: int = 0         # lattice-node updates of all runs of the search
    done: bool = False
    outside: str = ""        # "below" / "above" (Ca_cr outside the window) or "failed"

    @property
    def ca_cr(self):
        return 0.5 * (self.lo + self.hi)


def lattice_runner(precision: str = "fp32", log=None, **sim_kw):
    """Default run function of bisect: full simulations, one batch per round.
    Returns ([(broken, status, node updates)], seconds).  ``run.rounds`` lists
    (runs, node updates, seconds) per round."""
    def run(specs):
        if log:
            log(f" round of {len(specs)} runs")
        res, sec = simulate(specs, precision, progress=log, **sim_kw)
        out = [(r.broken, r.status, r.steps * r.params["nx"] * r.params["ny"] * r.params["nz"])
               for r in res]
        run.rounds.append((len(specs), sum(o[2] for o in out), sec))
        return out, sec
    run.rounds = []
    return run


def bisect(searches, tol: float = 0.02, run=None, max_rounds: int = 12):
    """Bisection in Ca for every search at once (each round's runs advance as
    one batch).  Per round and search: the unverified bracket ends are
    simulated together with the midpoint (speculatively: the midpoint result
    is discarded when an end check fails; a search with speculate=False runs
    only its unverified ends until both hold).  A lower end at hard_lo is taken as
    stable without a run (the bottom of the search window) while the search
    narrows; if the final bracket still rests on it, hard_lo is run once to
    verify it, and a break there ends the search as "below".  A failed end
    check moves the bracket outward by twice its width, clipped to the hard
    window: lo broken -> [lo - 2w, lo] (lo now a verified broken end);
    hi stable -> [hi, hi + 2w].  A run with a non-zero status ends its search
    as "failed".  Returns (searches, seconds, rounds).
    """
    run = run or lattice_runner()
    tol = tol * (1.0 + 1e-9)      # a bracket of width tol (up to rounding) is final
    total, rounds = 0.0, 0
    for s in searches:
        s.lo = max(s.lo, s.hard_lo)
        s.hi = min(s.hi, s.hard_hi)
        if s.lo <= s.hard_lo + 1e-12:
            s.lo, s.lo_ok, s.lo_assumed = s.hard_lo, True, True
    while rounds < max_rounds:
        todo, specs = [], []
        for s in searches:
            if s.done:
                continue
            if s.lo_ok and s.hi_ok and s.hi - s.lo <= tol:
                if s.lo_assumed:
                    todo.append((s, "lo", s.lo))     # verify the window's bottom once
                else:
                    s.done = True
                continue
            if not s.lo_ok:
                todo.append((s, "lo", s.lo))
            if not s.hi_ok:
                todo.append((s, "hi", s.hi))
            if s.hi - s.lo > tol and ((s.lo_ok and s.hi_ok) or s.speculate):
                todo.append((s, "mid", 0.5 * (s.lo + s.hi)))
        if not todo:
            break
        for s, _, ca in todo:
            specs.append(RunSpec(s.R, s.c, ca, s.De, s.lam, s.L2, s.fraction))
        outcomes, sec = run(specs)
        total += sec
        rounds += 1
        by_search = {}
        for (s, what, ca), out in zip(todo, outcomes):
            broken, status = out[0], out[1]
            s.runs += 1
            s.updates += out[2] if len(out) > 2 else 0
            by_search.setdefault(id(s), (s, {}))[1][what] = (ca, broken, status)
        for s, res in by_search.values():
            s.rounds += 1
            if any(st != 0 for _, _, st in res.values()):
                s.done, s.outside = True, "failed"
                continue
            moved = False
            if "lo" in res:
                ca, broken, _ = res["lo"]
                s.lo_assumed = False
                if not broken:
                    s.lo_ok = True
                elif ca <= s.hard_lo + 1e-12:
                    s.done, s.outside = True, "below"
                    continue
                else:
                    w = s.hi - s.lo
                    s.hi, s.hi_ok = ca, True
                    s.lo = max(s.hard_lo, ca - 2.0 * w)
                    s.lo_ok = s.lo <= s.hard_lo + 1e-12
                    moved = True
            if "hi" in res and not moved:
                ca, broken, _ = res["hi"]
                if broken:
                    s.hi_ok = True
                elif ca >= s.hard_hi - 1e-12:
                    s.done, s.outside = True, "above"
                    continue
                else:
                    w = s.hi - s.lo
                    s.lo, s.lo_ok, s.lo_assumed = ca, True, False
                    s.hi, s.hi_ok = min(s.hard_hi, ca + 2.0 * w), False
                    moved = True
            if "mid" in res and not moved:
                ca, broken, _ = res["mid"]
                if broken:
                    s.hi, s.hi_ok = ca, True
                else:
                    s.lo, s.lo_ok, s.lo_assumed = ca, True, False
        for s in searches:
            if not s.done and s.lo_ok and s.hi_ok and s.hi - s.lo <= tol and not s.lo_assumed:
                s.done = True
    return searches, total, rounds
