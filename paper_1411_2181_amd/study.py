"""Surrogate study: generate runs with the batched solver, train the network
on them, and compare surrogate-bracketed Ca_cr searches with plain
bisection on the same GPU.

    python -m paper_1411_2181_amd.study OUT.json [--runs 600] [--queries 32]

Workload readings (the reachable-parameter window of the lattice model):
R ~ U[12, 16] (break-up within the reachable Ca needs R >~ 16: the Reynolds
number at the wall-speed cap grows with R), lambda from {0.5, 0.75} (a droplet
tau of 1.5 or more dissolves the droplet at this coupling; lambda 1 and 2 are
outside the window), confinement c in {0.3, 0.5, 0.7}, De in {0, 0.5, 1, 2},
L^2 in {100, 400}, polymer fraction in {0.2, 0.4}; Ca ~ U[0.03, Ca_max],
Ca_max the value at the U_w = 0.19 wall-speed cap.  Each run lasts 8000 steps
(break-up, when it happens, does so by ~8000 steps) and is checked for
break-up every 1000 steps.  Query triples use R = 16.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import workloads as WL

from . import sweep
from .surrogate import Surrogate


def sample_specs(n: int, base_seed: int = 98765):
    specs = []
    for k in range(n):
        d = WL.surrogate_sampler(k, base_seed)
        rng = np.random.default_rng(d["seed"] + 17)
        R = float(rng.uniform(12.0, 16.0))
        lam = 0.5 if d["lam"] <= 0.5 else 0.75
        hi = sweep.ca_max(R, d["confinement"], lam, d["De"], d["polymer_fraction"])
        Ca = float(rng.uniform(0.03, hi))
        specs.append(sweep.RunSpec(R, d["confinement"], Ca, d["De"], lam, d["L2"],
                                   d["polymer_fraction"]))
    return specs


def generate(specs, chunk: int = 80, steps: int = 8000, log=print):
    rows, secs, updates = [], 0.0, 0
    for i in range(0, len(specs), chunk):
        part = specs[i:i + chunk]
        res, sec = sweep.simulate(part, "fp32", t_end=steps, every=1000)
        secs += sec
        for r in res:
            n = r.params["nx"] * r.params["ny"] * r.params["nz"]
            updates += n * r.steps
            rows.append(dict(inputs=r.spec.inputs(), D=r.D, theta=r.theta, broken=bool(r.broken),
                             status=r.status, steps=r.steps, Lp_max=r.Lp_max))
        log(f"generated {i + len(part)}/{len(specs)} runs, {secs:.1f} s, "
            f"{updates / secs / 1e6:.0f} MLUPS (batched FP32)")
    return rows, secs, updates


def query_searches(n: int, R: float = 16.0):
    out = []
    for q in WL.query_triples(n):
        lam = min(max(q["lam"], 0.5), 0.8)
        out.append(dict(De=q["De"], lam=lam, c=q["confinement"], R=R))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--runs", type=int, default=320)
    ap.add_argument("--queries", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=3000)
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    report = {}

    # 1. training data from the solver itself
    specs = sample_specs(args.runs)
    rows, sec, upd = generate(specs, log=log)
    ok = [r for r in rows if r["status"] == 0]
    report["data"] = dict(runs=len(rows), usable=len(ok), broken=sum(r["broken"] for r in ok),
                          seconds=sec, updates=upd, mlups=upd / sec / 1e6)
    X = np.array([r["inputs"] for r in ok])
    D = np.array([r["D"] for r in ok])
    TH = np.array([r["theta"] for r in ok])
    BR = np.array([r["broken"] for r in ok], dtype=float)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(ok))
    nte = max(1, len(ok) // 10)
    te, tr = perm[:nte], perm[nte:]

    # 2. train on the GPU with the project's kernels
    sg = Surrogate(batch_max=max(4096, len(tr)), seed=1)
    t0 = time.perf_counter()
    losses = sg.fit(X[tr], D[tr], TH[tr], BR[tr], epochs=args.epochs, lr=2e-3)
    report["train"] = dict(rows=int(tr.size), epochs=args.epochs, loss_first=losses[0],
                           loss_last=losses[-1], seconds=time.perf_counter() - t0)
    pD, pT, pB = sg.predict(X[te])
    unb = BR[te] < 0.5
    report["holdout"] = dict(
        rows=int(te.size),
        mae_D=float(np.mean(np.abs(pD[unb] - D[te][unb]))) if unb.any() else None,
        mae_theta_deg=float(np.mean(np.abs(pT[unb] - TH[te][unb]))) if unb.any() else None,
        breakup_accuracy=float(np.mean((pB >= 0.5) == (BR[te] > 0.5))))
    log(json.dumps(report))

    # 3. Ca_cr searches: plain bisection vs surrogate-proposed brackets
    qs = query_searches(args.queries)
    plain = [sweep.Search(q["De"], q["lam"], q["c"], q["R"], 0.0, 1e9) for q in qs]
    plain, t_plain, r_plain = sweep.bisect(plain, tol=0.02, verify_ends=False, t_end=8000)
    log(f"plain bisection: {t_plain:.1f} s, {r_plain} rounds, {sum(s.runs for s in plain)} runs")
    prop = []
    for q in qs:
        hi = sweep.ca_max(q["R"], q["c"], q["lam"], q["De"])
        b = sg.propose(q["De"], q["lam"], q["c"], 0.02, hi)
        lo_b, hi_b = b if b is not None else (0.02, hi)
        prop.append(sweep.Search(q["De"], q["lam"], q["c"], q["R"], lo_b, hi_b))
    prop, t_sg, r_sg = sweep.bisect(prop, tol=0.02, verify_ends=True, t_end=8000)
    log(f"surrogate-bracketed: {t_sg:.1f} s, {r_sg} rounds, {sum(s.runs for s in prop)} runs")
    rows_q = []
    agree = 0
    comparable = 0
    for q, a, b in zip(qs, plain, prop):
        rq = dict(q, plain=a.ca_cr, plain_outside=a.outside, surrogate=b.ca_cr,
                  surrogate_outside=b.outside, runs_plain=a.runs, runs_surrogate=b.runs)
        if not b.outside and a.lo > a.hard_lo + 1e-9 and a.hi < a.hard_hi - 1e-9:
            comparable += 1
            agree += abs(a.ca_cr - b.ca_cr) <= 0.02
        rows_q.append(rq)
    report["search"] = dict(
        queries=len(qs), tol=0.02,
        plain=dict(seconds=t_plain, rounds=r_plain, runs=sum(s.runs for s in plain),
                   sweeps_per_hour=len(qs) / t_plain * 3600),
        surrogate=dict(seconds=t_sg, rounds=r_sg, runs=sum(s.runs for s in prop),
                       sweeps_per_hour=len(qs) / t_sg * 3600,
                       verified_first_try=sum(1 for s in prop if s.runs <= 3)),
        comparable=comparable, agree_within_0p02=agree, rows=rows_q)

    # 4. plain FP64 one-run-at-a-time bisection on two triples (extrapolated)
    t64 = 0.0
    n64 = 0
    for q in qs[:2]:
        s = [sweep.Search(q["De"], q["lam"], q["c"], q["R"], 0.0, 1e9)]
        _, t, _ = sweep.bisect(s, tol=0.02, verify_ends=False, precision="fp64", t_end=8000)
        t64 += t
        n64 += 1
    report["search"]["plain_fp64_single"] = dict(
        triples_timed=n64, seconds=t64, sweeps_per_hour=n64 / t64 * 3600)
    sg.close()
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    log(json.dumps(report["search"]["plain"]))
    log(json.dumps(report["search"]["surrogate"]))
    log(json.dumps(report["search"]["plain_fp64_single"]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
