"""Surrogate study: runs from the batched solver train the network, which
then proposes Ca_cr brackets; plain bisection on the same GPU is the
reference.

    python -m paper_1411_2181_amd.study generate DATA.json [--runs 160] [--skip 0] [--near D1.json]
    python -m paper_1411_2181_amd.study search OUT.json --data DATA.json[,DATA2.json] \
        [--queries 32] [--fp64-queries 1] [--precision fp32|fp16s] [--extend-to N] \
        [--only I,J,...] [--plain-only]
    python -m paper_1411_2181_amd.study elongation OUT.json --search SEARCH.json [--queries 4]
    python -m paper_1411_2181_amd.study fp64 OUT.json [--queries 4] [--compare SEARCH.json]
    python -m paper_1411_2181_amd.study scan OUT.json --De 1.2 --c 0.63 --fraction 0.2 \
        --ca 0.18,0.2,0.22 [--t-end 16000]

Study window (the part of parameter space where the droplet breaks at a
reachable capillary number and keeps its volume): R = 24 (Reynolds number
5-7 at the wall-speed cap, where break-up sets in at Ca ~ 0.2), confinement
c ~ U[0.45, 0.65], De in {0, 0.5, 1, 2}, L^2 in {100, 400}, polymer fraction
f in {0.2, 0.4}, droplet viscoelastic.  The droplet's solvent is held at
tau_A = TAU_DROP next to the tau = 1.5 matrix: with the velocity-shift
forcing a droplet whose tau is lower takes up matrix component and swells
(by 36-65 % over 16000 steps at tau_A = 0.86-1.1), at 1.3 it keeps its
volume.  The viscosity ratio is therefore lambda = LAM_N / (1 - f)
(LAM_N = 0.8 for a Newtonian droplet).  Ca ~ U[CA_LO, Ca_max], Ca_max the
value at the U_w = 0.19 cap.  Each run lasts up to T_END steps and is checked
for break-up every EVERY steps (a run stops once it breaks).

Training data: a first batch from the window sampler, then (``--near``) a
batch placed where the network trained on the first one is uncertain.

Searches: tolerance 0.02 (Ca_cr located within +-0.01), window
[CA_LO, Ca_max] with CA_LO taken as stable.  Plain bisection starts from the
window; the surrogate's search starts from the network's bracket (centred
where its break-up probability crosses 1/2, at least +-0.02 wide) and falls
back outward when a bracket end fails (sweep.bisect).  Both advance every query's runs of a round
as one batch (FP32 or FP16S storage).  A run lasts T_END steps; a droplet still
stretching at T_END runs on, check by check, up to ``--extend-to`` steps
(default 2 T_END; sweep.simulate), which keeps slow binary break-ups just
below the onset of ternary break-up from being taken as stable.  The plain FP64 one-run-at-a-time variant is timed on
``--fp64-queries`` triples.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as WL

from . import sweep
from .surrogate import Surrogate

CA_LO = 0.12
LAM_N = 0.8          # Newtonian droplet: tau_A = 0.5 + 3 LAM_N eta_M = 1.3 at tau_M = 1.5
T_END = 16000
EVERY = 2000
TOL = 0.02


def window_lambda(De: float, fraction: float):
    """Viscosity ratio and polymer fraction that keep the droplet's solvent
    at tau_A = 1.3: lambda = LAM_N/(1 - f) with polymer, LAM_N without."""
    if De <= 0.0:
        return LAM_N, 0.0
    return LAM_N / (1.0 - fraction), fraction


def sample_specs(n: int, base_seed: int = 98765):
    specs = []
    for k in range(n):
        d = WL.surrogate_window_sampler(k, base_seed)
        lam, f = window_lambda(d["De"], d["polymer_fraction"])
        hi = sweep.ca_max(d["R"], d["confinement"], lam, d["De"], f)
        Ca = CA_LO + d["u"] * (hi - CA_LO)
        specs.append(sweep.RunSpec(d["R"], d["confinement"], Ca, d["De"], lam, d["L2"], f))
    return specs


def generate(specs, chunk: int = 20, log=print, save=None):
    rows, secs, updates = [], 0.0, 0
    for i in range(0, len(specs), chunk):
        part = specs[i:i + chunk]
        res, sec = sweep.simulate(part, "fp32", t_end=T_END, every=EVERY, progress=log)
        secs += sec
        for r in res:
            n = r.params["nx"] * r.params["ny"] * r.params["nz"]
            updates += n * r.steps
            rows.append(dict(inputs=r.spec.inputs(), D=r.D, theta=r.theta, broken=bool(r.broken),
                             step_break=r.step_break, status=r.status, steps=r.steps,
                             Lp_max=r.Lp_max, R=r.spec.R))
        log(f"generated {i + len(part)}/{len(specs)} runs, {secs:.1f} s, "
            f"{updates / secs / 1e6:.0f} MLUPS (batched FP32), "
            f"{sum(r['broken'] for r in rows)} broken")
        if save:
            save(rows, secs, updates)
    return rows, secs, updates


def query_searches(n: int):
    out = []
    for q in WL.query_window(n):
        lam, f = window_lambda(q["De"], q["polymer_fraction"])
        out.append(dict(De=q["De"], lam=lam, c=q["confinement"], R=q["R"], L2=q["L2"], fraction=f))
    return out


def window(q):
    return CA_LO, sweep.ca_max(q["R"], q["c"], q["lam"], q["De"], q["fraction"])


def single_runner(precision: str, log=None, extend_to: int = 0):
    """One run at a time (no batching): the plain reference path (with the
    batched searches' horizon extension)."""
    def run(specs):
        out, total = [], 0.0
        for sp in specs:
            res, sec = sweep.simulate([sp], precision, t_end=T_END, every=EVERY, progress=log,
                                      extend_to=extend_to)
            total += sec
            r = res[0]
            out.append((r.broken, r.status, r.steps * r.params["nx"] * r.params["ny"] * r.params["nz"]))
        return out, total
    return run


def _plain(o):
    """JSON form of NumPy scalars and tuples inside the report."""
    if isinstance(o, np.generic):
        return o.item()
    raise TypeError(type(o))


def near_boundary_specs(n, data_paths, base_seed=55555, pool=4000, band=(0.15, 0.85), log=print):
    """Active-learning batch: train the network on earlier runs, then keep,
    in sampler order, the first n window samples whose predicted break-up
    probability lies in ``band`` (where the boundary is still uncertain)."""
    data = load_data(data_paths)
    ok = [r for r in data["rows"] if r["status"] == 0]
    sg = Surrogate(batch_max=max(4096, len(ok), pool), seed=1)
    sg.fit(np.array([r["inputs"] for r in ok]), np.array([r["D"] for r in ok]),
           np.array([r["theta"] for r in ok]), np.array([r["broken"] for r in ok], dtype=float),
           epochs=3000, lr=2e-3)
    cands = sample_specs(pool, base_seed)
    p = sg.predict(np.array([sp.inputs() for sp in cands]))[2]
    sg.close()
    keep = [sp for sp, pk in zip(cands, p) if band[0] < pk < band[1]][:n]
    log(f"near-boundary batch: {len(keep)} of {pool} candidates with p in {band}")
    return keep


def cmd_generate(args, log):
    if args.near:
        specs = near_boundary_specs(args.runs, args.near.split(","), log=log)
    else:
        specs = sample_specs(args.runs + args.skip)[args.skip:]

    def save(rows, sec, upd):
        with open(args.out, "w") as fh:
            json.dump(dict(window=dict(R=24.0, ca_lo=CA_LO, t_end=T_END, every=EVERY),
                           first_run=args.skip, near=args.near, seconds=sec, updates=upd,
                           rows=rows), fh, indent=1, default=_plain)

    generate(specs, log=log, save=save)
    return 0


def load_data(paths):
    """Merge generate outputs (each a slice of the same sampler sequence)."""
    rows, sec, upd = [], 0.0, 0
    for p in paths:
        with open(p) as fh:
            d = json.load(fh)
        rows += d["rows"]
        sec += d["seconds"]
        upd += d["updates"]
    return dict(rows=rows, seconds=sec, updates=upd)


def cmd_search(args, log):
    data = load_data(args.data.split(","))
    rows = data["rows"]
    ok = [r for r in rows if r["status"] == 0]
    report = dict(data=dict(runs=len(rows), usable=len(ok), broken=sum(r["broken"] for r in ok),
                            failed=len(rows) - len(ok), seconds=data["seconds"],
                            mlups=data["updates"] / data["seconds"] / 1e6))
    X = np.array([r["inputs"] for r in ok])
    D = np.array([r["D"] for r in ok])
    TH = np.array([r["theta"] for r in ok])
    BR = np.array([r["broken"] for r in ok], dtype=float)
    if args.holdout:
        # a separate set of runs (another slice of the sampler), never trained on
        hold = [r for r in load_data(args.holdout.split(","))["rows"] if r["status"] == 0]
        n0 = len(ok)
        X = np.concatenate([X, np.array([r["inputs"] for r in hold])])
        D = np.concatenate([D, np.array([r["D"] for r in hold])])
        TH = np.concatenate([TH, np.array([r["theta"] for r in hold])])
        BR = np.concatenate([BR, np.array([r["broken"] for r in hold], dtype=float)])
        tr, te = np.arange(n0), np.arange(n0, n0 + len(hold))
    else:
        rng = np.random.default_rng(0)
        perm = rng.permutation(len(ok))
        nte = max(1, len(ok) // 10)
        te, tr = perm[:nte], perm[nte:]

    # train on the GPU with the project's kernels
    sg = Surrogate(batch_max=max(4096, len(ok)), seed=1)
    t0 = time.perf_counter()
    losses = sg.fit(X[tr], D[tr], TH[tr], BR[tr], epochs=args.epochs, lr=2e-3)
    report["train"] = dict(rows=int(tr.size), epochs=args.epochs, loss_first=losses[0],
                           loss_last=losses[-1], seconds=time.perf_counter() - t0)
    pD, pT, pB = sg.predict(X[te])
    unb = BR[te] < 0.5
    report["holdout"] = dict(
        rows=int(te.size), broken=int(BR[te].sum()),
        mae_D=float(np.mean(np.abs(pD[unb] - D[te][unb]))) if unb.any() else None,
        mae_theta_deg=float(np.mean(np.abs(pT[unb] - TH[te][unb]))) if unb.any() else None,
        breakup_accuracy=float(np.mean((pB >= 0.5) == (BR[te] > 0.5))))
    log(json.dumps(report))
    # refit on every usable training row for the searches (the held-out set
    # of --holdout stays out)
    sg.close()
    sg = Surrogate(batch_max=max(4096, len(ok)), seed=1)
    keep = tr if args.holdout else np.arange(len(ok))
    sg.fit(X[keep], D[keep], TH[keep], BR[keep], epochs=args.epochs, lr=2e-3)

    qs = query_searches(args.queries)
    if args.only:
        qs = [qs[int(i)] for i in args.only.split(",")]
    ext = dict(extend_to=args.extend_to) if args.extend_to else {}

    def plain_searches():
        out = []
        for q in qs:
            lo, hi = window(q)
            out.append(sweep.Search(q["De"], q["lam"], q["c"], q["R"], lo, hi, hard_lo=lo, hard_hi=hi,
                                    L2=q["L2"], fraction=q["fraction"]))
        return out

    prec = args.precision
    # plain bisection, batched
    run_plain = sweep.lattice_runner(prec, log=log, t_end=T_END, every=EVERY, **ext)
    plain, t_plain, r_plain = sweep.bisect(plain_searches(), tol=TOL, run=run_plain)
    log(f"plain bisection ({prec}): {t_plain:.1f} s, {r_plain} rounds, {sum(s.runs for s in plain)} runs")
    # the plain search's brackets so far (the file is rewritten with the whole report at the end)
    with open(args.out, "w") as fh:
        json.dump(dict(report, partial=dict(plain_seconds=t_plain, plain_rounds=r_plain, rows=[
            dict(q, plain=dict(ca_cr=a.ca_cr, bracket=[a.lo, a.hi], outside=a.outside, runs=a.runs))
            for q, a in zip(qs, plain)])), fh, indent=1, default=_plain)

    # surrogate-proposed brackets, batched FP32
    prop, proposals = [], []
    for q in qs:
        lo, hi = window(q)
        b = sg.propose(q["De"], q["lam"], q["c"], lo, hi, tol=TOL)
        proposals.append(b)
        # no predicted crossing: check the top of the window first (one run);
        # if it breaks after all, the search goes on as plain bisection
        blo, bhi = b if b is not None else (lo, hi)
        prop.append(sweep.Search(q["De"], q["lam"], q["c"], q["R"], blo, bhi, hard_lo=lo, hard_hi=hi,
                                 L2=q["L2"], fraction=q["fraction"], speculate=b is not None))
    run_sg = sweep.lattice_runner(prec, log=log, t_end=T_END, every=EVERY, **ext)
    if args.plain_only:
        prop = []
    prop, t_sg, r_sg = sweep.bisect(prop, tol=TOL, run=run_sg) if prop else ([], 0.0, 0)
    log(f"surrogate-bracketed ({prec}): {t_sg:.1f} s, {r_sg} rounds, {sum(s.runs for s in prop)} runs")

    rows_q, agree, comparable = [], 0, 0
    for k, (q, a, pb) in enumerate(zip(qs, plain, proposals)):
        row = dict(q, window=list(window(q)), proposal=pb,
                   plain=dict(ca_cr=a.ca_cr, bracket=[a.lo, a.hi], outside=a.outside,
                              runs=a.runs, rounds=a.rounds, updates=a.updates))
        if prop:
            b = prop[k]
            row["surrogate"] = dict(ca_cr=b.ca_cr, bracket=[b.lo, b.hi], outside=b.outside,
                                    runs=b.runs, rounds=b.rounds, updates=b.updates)
            if a.outside == b.outside:
                comparable += 1
                agree += (a.outside != "" or abs(a.ca_cr - b.ca_cr) <= TOL)
        rows_q.append(row)
    # sweeps per hour at saturation: with many queries in flight the GPU is
    # full and time goes as lattice updates, not as rounds.  The saturated
    # rate is that of the largest batch either search ran (the plain search's
    # first round: two runs per query).
    big = max(run_plain.rounds + run_sg.rounds)
    rate = big[1] / big[2]
    upd_plain = sum(s.updates for s in plain)
    upd_sg = sum(s.updates for s in prop)
    report["search"] = dict(
        queries=len(qs), tol=TOL, t_end=T_END, extend_to=args.extend_to, precision=prec,
        only=args.only,
        saturated_batch=dict(runs=big[0], updates=big[1], seconds=big[2]),
        plain=dict(seconds=t_plain, rounds=r_plain, runs=sum(s.runs for s in plain),
                   updates=upd_plain, sweeps_per_hour=len(qs) / t_plain * 3600,
                   sweeps_per_hour_saturated=len(qs) / (upd_plain / rate) * 3600),
        surrogate=dict(seconds=t_sg, rounds=r_sg, runs=sum(s.runs for s in prop),
                       updates=upd_sg, sweeps_per_hour=len(qs) / t_sg * 3600,
                       sweeps_per_hour_saturated=len(qs) / (upd_sg / rate) * 3600,
                       first_round_hits=sum(1 for s in prop if s.rounds == 1 and s.outside == ""))
        if prop else None,
        batched_rate_mlups=rate / 1e6,
        same_outcome=comparable, agree_within_tol=agree, rows=rows_q)

    # plain FP64, one run at a time, on the first triples
    t64, n64, runs64 = 0.0, 0, 0
    for q in qs[:args.fp64_queries]:
        lo, hi = window(q)
        s64 = [sweep.Search(q["De"], q["lam"], q["c"], q["R"], lo, hi, hard_lo=lo, hard_hi=hi,
                            L2=q["L2"], fraction=q["fraction"])]
        s64, t, _ = sweep.bisect(s64, tol=TOL, run=single_runner("fp64", log, getattr(args, "extend_to", 0)))
        t64 += t
        n64 += 1
        runs64 += s64[0].runs
        log(f"fp64 single: query {n64} {t:.1f} s, {s64[0].runs} runs, Ca_cr {s64[0].ca_cr:.3f} "
            f"({s64[0].outside or 'inside'}); batched plain {plain[n64 - 1].ca_cr:.3f}")
    if n64:
        report["search"]["plain_fp64_single"] = dict(triples_timed=n64, seconds=t64, runs=runs64,
                                                     sweeps_per_hour=n64 / t64 * 3600)
    sg.close()
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1, default=_plain)
    for k in ("plain", "surrogate", "plain_fp64_single"):
        if k in report["search"]:
            log(k + " " + json.dumps(report["search"][k]))
    log(f"same outcome {comparable}/{len(qs)}, agree within tol {agree}")
    return 0


def cmd_elongation(args, log):
    """Elongation histories L_p(t)/2R of a pre-critical (stable) and a
    post-critical (breaking) run on each side of a located Ca_cr, the
    counterpart of the paper's Fig. 4(b), with the number of daughter drops
    at break-up (two: binary; three or more: multiple necking, Section 3) and
    their sizes (the spread, (largest - smallest) / mean, measures how far
    from monodisperse the daughters are)."""
    with open(args.search) as fh:
        found = [r for r in json.load(fh)["search"]["rows"] if r["plain"]["outside"] == ""]
    specs, tags = [], []
    for q in found[:args.queries]:
        lo, hi = q["plain"]["bracket"]
        for side, ca in (("pre", lo), ("post", hi)):
            specs.append(sweep.RunSpec(q["R"], q["c"], ca, q["De"], q["lam"], q.get("L2", 100.0),
                                       q["fraction"]))
            tags.append(dict(De=q["De"], lam=q["lam"], c=q["c"], R=q["R"], Ca=ca, side=side))
    res, sec = sweep.simulate(specs, "fp32", t_end=T_END, every=args.every, progress=log)
    rows = []
    for t, r in zip(tags, res):
        tem = r.info["tau_em"]
        hist = [dict(step=h[0], t_over_tau_em=h[0] / tem, D=h[1], theta=h[2],
                     Lp_over_2R=h[3] / (2 * t["R"]), pieces=h[4]) for h in r.history]
        sizes = r.pieces
        spread = (max(sizes) - min(sizes)) / (sum(sizes) / len(sizes)) if sizes else None
        rows.append(dict(t, broken=r.broken, step_break=r.step_break,
                         daughters=r.history[-1][4] if r.broken else 1,
                         daughter_nodes=sizes, daughter_spread=spread,
                         Lp_max_over_2R=max(h["Lp_over_2R"] for h in hist), tau_em=tem,
                         history=hist))
        log(f"{t['side']:4s} Ca={t['Ca']:.3f} De={t['De']:.2f} lam={t['lam']:.2f} c={t['c']:.3f}: "
            f"{'breaks at %d into %d %s' % (r.step_break, rows[-1]['daughters'], sizes) if r.broken else 'stable'}, "
            f"max Lp/2R {rows[-1]['Lp_max_over_2R']:.2f}")
    with open(args.out, "w") as fh:
        json.dump(dict(seconds=sec, every=args.every, t_end=T_END, rows=rows), fh, indent=1,
                  default=_plain)
    return 0


def cmd_fp64(args, log):
    """Plain bisection in FP64, one run at a time (the reference path), on
    the first --queries query triples; with --compare, each located Ca_cr is
    set beside the batched plain search's for the same triple."""
    qs = query_searches(args.queries)
    ref = None
    if args.compare:
        with open(args.compare) as fh:
            ref = json.load(fh)["search"]["rows"]
    rows, total, runs = [], 0.0, 0
    for k, q in enumerate(qs):
        lo, hi = window(q)
        s64 = [sweep.Search(q["De"], q["lam"], q["c"], q["R"], lo, hi, hard_lo=lo, hard_hi=hi,
                            L2=q["L2"], fraction=q["fraction"])]
        s64, t, _ = sweep.bisect(s64, tol=TOL, run=single_runner("fp64", log, getattr(args, "extend_to", 0)))
        a = s64[0]
        total += t
        runs += a.runs
        row = dict(q, seconds=t, runs=a.runs, ca_cr=a.ca_cr, bracket=[a.lo, a.hi], outside=a.outside)
        if ref is not None:
            r = ref[k]["plain"]
            row["batched_plain"] = dict(ca_cr=r["ca_cr"], bracket=r["bracket"], outside=r["outside"])
            row["same_bracket"] = (r["outside"] == a.outside and abs(r["bracket"][0] - a.lo) < 1e-12
                                   and abs(r["bracket"][1] - a.hi) < 1e-12)
        rows.append(row)
        log(f"fp64 single: query {k + 1} {t:.1f} s, {a.runs} runs, Ca_cr {a.ca_cr:.3f} "
            f"({a.outside or 'inside'})" + (f", same bracket as batched: {row['same_bracket']}"
                                              if ref is not None else ""))
        # the report so far after every query (a long run keeps what it finished)
        out = dict(queries=len(rows), tol=TOL, t_end=T_END,
                   extend_to=getattr(args, "extend_to", 0), seconds=total, runs=runs,
                   sweeps_per_hour=len(rows) / total * 3600, rows=rows)
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1, default=_plain)
    log(f"fp64 single: {len(qs)} queries, {total:.1f} s, {runs} runs, "
        f"{out['sweeps_per_hour']:.1f} sweeps per hour")
    return 0


def cmd_scan(args, log):
    """Break-up against Ca at one (De, lambda, c) point: every Ca of the list
    runs for up to --t-end steps in one batch, checked every --every steps,
    with its break-up step, daughter sizes and elongation history.  Shows
    where break-up is not monotonic in Ca (a stable window above a breaking
    Ca), which bisection cannot see."""
    lam, f = window_lambda(args.De, args.fraction)
    cas = [float(v) for v in args.ca.split(",")]
    specs = [sweep.RunSpec(args.R, args.c, ca, args.De, lam, args.L2, f) for ca in cas]
    res, sec = sweep.simulate(specs, args.precision, t_end=args.t_end, every=args.every, progress=log)
    rows = []
    for ca, r in zip(cas, res):
        tem = r.info["tau_em"]
        hist = [dict(step=h[0], D=h[1], theta=h[2], Lp_over_2R=h[3] / (2 * args.R), pieces=h[4])
                for h in r.history]
        rows.append(dict(Ca=ca, broken=r.broken, step_break=r.step_break, status=r.status,
                         t_break_over_tau_em=(r.step_break / tem) if r.broken else None,
                         daughter_nodes=r.pieces, Lp_max_over_2R=max(h["Lp_over_2R"] for h in hist),
                         history=hist))
        log(f"Ca={ca:.3f}: " + (f"breaks at {r.step_break} into {len(r.pieces)} {r.pieces}" if r.broken
                                 else "stable") + f", max Lp/2R {rows[-1]['Lp_max_over_2R']:.2f}")
    out = dict(De=args.De, lam=lam, fraction=f, c=args.c, R=args.R, L2=args.L2,
               precision=args.precision, t_end=args.t_end, every=args.every, seconds=sec,
               tau_em=res[0].info["tau_em"], rows=rows)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1, default=_plain)
    return 0


# Matrix solvent relaxation time per mode in cmd_modes: Newtonian and
# droplet-viscoelastic runs use the search window's; the matrix-viscoelastic
# droplet (total viscosity of the matrix solvent + polymer, lambda = 1) needs
# a lower matrix solvent tau so the droplet's tau stays in the calibrated
# (Laplace-consistent) range.
MODE_TAU_MATRIX = {"N": 1.5, "DV": 1.5, "MV": 0.98}


def cmd_modes(args, log):
    """Newtonian, droplet-viscoelastic and matrix-viscoelastic droplets at
    the same Ca, confinement 2R/W and viscosity ratio (lambda = 1 in the
    total viscosities, the paper's choice in Section 3), for each De of the
    list: elongation histories L_p(t)/2R, break-up step and daughter sizes,
    the counterpart of the paper's Fig. 4 (its Section 3 compares the three
    at 2R/W = 0.78).  All runs advance as one batch, up to --t-end steps,
    extended to --extend-to for runs still elongating."""
    specs, tags = [], []
    for ca in (float(v) for v in args.ca.split(",")):
        specs.append(sweep.RunSpec(args.R, args.c, ca, 0.0, 1.0, args.L2, args.fraction, phase="N",
                                   tau_matrix=MODE_TAU_MATRIX["N"]))
        tags.append(dict(mode="N", Ca=ca, De=0.0))
        for De in (float(v) for v in args.De.split(",")):
            for mode in ("DV", "MV"):
                specs.append(sweep.RunSpec(args.R, args.c, ca, De, 1.0, args.L2, args.fraction,
                                           phase=mode, tau_matrix=MODE_TAU_MATRIX[mode]))
                tags.append(dict(mode=mode, Ca=ca, De=De))
    res, sec = sweep.simulate(specs, args.precision, t_end=args.t_end, every=args.every,
                              progress=log, extend_to=args.extend_to)
    rows = []
    for t, r in zip(tags, res):
        tem = r.info["tau_em"]
        hist = [dict(step=h[0], t_over_tau_em=h[0] / tem, D=h[1], theta=h[2],
                     Lp_over_2R=h[3] / (2 * args.R), pieces=h[4]) for h in r.history]
        rows.append(dict(t, tau=list(r.params["tau"]), tau_P=list(r.params["tau_P"]),
                         u_wall=r.params["u_wall"], tau_em=tem, broken=r.broken,
                         step_break=r.step_break, status=r.status, steps=r.steps,
                         t_break_over_tau_em=(r.step_break / tem) if r.broken else None,
                         daughter_nodes=r.pieces,
                         Lp_max_over_2R=max(h["Lp_over_2R"] for h in hist), history=hist))
        log(f"{t['mode']:2s} Ca={t['Ca']:.3f} De={t['De']:.2f}: "
            + (f"breaks at {r.step_break} into {len(r.pieces)} {r.pieces}" if r.broken else "stable")
            + f", max Lp/2R {rows[-1]['Lp_max_over_2R']:.2f}")
    out = dict(c=args.c, R=args.R, L2=args.L2, fraction=args.fraction, lam=1.0,
               tau_matrix=MODE_TAU_MATRIX, precision=args.precision, t_end=args.t_end,
               extend_to=args.extend_to, every=args.every, seconds=sec, rows=rows)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1, default=_plain)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("out")
    g.add_argument("--runs", type=int, default=160)
    g.add_argument("--skip", type=int, default=0, help="start at this run of the sampler sequence")
    g.add_argument("--near", default="", help="earlier generate outputs: place the runs where "
                                              "the network trained on them is uncertain")
    s = sub.add_parser("search")
    s.add_argument("out")
    s.add_argument("--data", required=True, help="comma-separated generate outputs")
    s.add_argument("--queries", type=int, default=32)
    s.add_argument("--holdout", default="", help="generate outputs held out of training "
                   "(scored only); without it 10 %% of --data is held out")
    s.add_argument("--epochs", type=int, default=3000)
    s.add_argument("--fp64-queries", type=int, default=1)
    s.add_argument("--precision", default="fp32", choices=["fp32", "fp16s"],
                   help="storage of the batched searches")
    s.add_argument("--extend-to", type=int, default=2 * T_END,
                   help="run a droplet still elongating at the horizon on, up to this step "
                        "(0: fixed horizon)")
    s.add_argument("--only", default="", help="comma-separated indices of the query triples")
    s.add_argument("--plain-only", action="store_true", help="skip the surrogate's search")
    e = sub.add_parser("elongation")
    e.add_argument("out")
    e.add_argument("--search", required=True, help="a search output (brackets of located Ca_cr)")
    e.add_argument("--queries", type=int, default=4)
    e.add_argument("--every", type=int, default=500)
    f64 = sub.add_parser("fp64")
    f64.add_argument("out")
    f64.add_argument("--queries", type=int, default=4)
    f64.add_argument("--compare", default="", help="a search output of the same query triples")
    f64.add_argument("--extend-to", type=int, default=2 * T_END,
                     help="horizon extension of runs still elongating (as in search); 0: off")
    k = sub.add_parser("scan")
    k.add_argument("out")
    k.add_argument("--De", type=float, required=True)
    k.add_argument("--c", type=float, required=True)
    k.add_argument("--fraction", type=float, default=0.4)
    k.add_argument("--L2", type=float, default=100.0)
    k.add_argument("--R", type=float, default=24.0)
    k.add_argument("--ca", required=True, help="comma-separated capillary numbers")
    k.add_argument("--t-end", type=int, default=T_END)
    k.add_argument("--every", type=int, default=500)
    k.add_argument("--precision", default="fp32", choices=["fp32", "fp16s"])
    m = sub.add_parser("modes")
    m.add_argument("out")
    m.add_argument("--c", type=float, default=0.78)
    m.add_argument("--R", type=float, default=24.0)
    m.add_argument("--ca", required=True, help="comma-separated capillary numbers")
    m.add_argument("--De", default="0.2,2", help="comma-separated Deborah numbers")
    m.add_argument("--fraction", type=float, default=0.4)
    m.add_argument("--L2", type=float, default=100.0)
    m.add_argument("--t-end", type=int, default=T_END)
    m.add_argument("--extend-to", type=int, default=2 * T_END)
    m.add_argument("--every", type=int, default=500)
    m.add_argument("--precision", default="fp32", choices=["fp32", "fp16s"])
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    cmd = {"generate": cmd_generate, "search": cmd_search, "elongation": cmd_elongation,
           "scan": cmd_scan, "fp64": cmd_fp64, "modes": cmd_modes}
    return cmd[args.cmd](args, log)


if __name__ == "__main__":
    sys.exit(main())
