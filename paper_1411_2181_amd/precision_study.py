"""Storage-precision study: FP32 and shift-stored FP16 populations against the
FP64 path (itself parity-checked against the oracle) on the two larger
droplet workloads.

    python -m paper_1411_2181_amd.precision_study OUT.json [--c3-steps 50000] \
        [--c3-lambdas 0.5,2] [--skip-c2]

* 192x96x64 (W = 64), R = 16, polymer in the droplet (L^2 = 100, fraction
  0.4), lambda = 1, De in {0.5, 1, 2} x Ca in {0.1, 0.2} (Ca = 0.3 needs a
  wall speed above the 0.19 cap at the calibrated sigma), 20000 steps: the
  six runs advance as one batch per precision.
* 512x256x128 (W = 128), R = 32, polymer in the matrix (L^2 = 400, De = 1,
  fraction 0.4), U_w = 0.1, lambda = 0.5 (tau_A = 4/3, tau_B = 1.5) and
  lambda = 2 (tau_A = 1.75, tau_B = 0.875: with 40 % of the matrix viscosity
  in the polymer, lambda = 2 puts the matrix solvent below the
  Laplace-calibrated tau window; every precision follows the same dynamics,
  which is what this comparison needs): deformation, orientation and the
  relative L2 error of the velocity field at checkpoints every 10000 steps.

Reported per result: |D - D_64|, |theta - theta_64|, velocity rel. L2, mass
drift per component.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbmve, physics

PRECISIONS = ("fp64", "fp32", "fp16s")


def c2_runs():
    runs, tags = [], []
    for De in (0.5, 1.0, 2.0):
        for Ca in (0.1, 0.2):
            p, info = physics.lattice_params(192, 96, 64, 16.0, Ca, De, 1.0, phase="DV",
                                             L2=100.0, fraction=0.4, tau_matrix=1.5, u_max=0.19)
            runs.append(p)
            tags.append(dict(De=De, Ca=Ca, u_wall=p["u_wall"], tau=p["tau"], tau_P=p["tau_P"][0]))
    return runs, tags


def c3_run(lam=0.5):
    import bench
    p, info = bench.workload_params()
    if lam != 0.5:
        # same wall speed, tau_P and polymer; droplet and matrix solvents set
        # for lambda = eta_A / eta_M with eta_M = eta_B / (1 - 0.4)
        tau_A = 1.75
        eta_A = physics.eta_of_tau(tau_A)
        eta_M = eta_A / lam
        tau_B = physics.tau_of_eta(0.6 * eta_M)
        p = dict(p, tau=(tau_A, tau_B), eta_P=(0.0, 0.4 * eta_M))
    return p, dict(lam=lam, u_wall=p["u_wall"], tau=p["tau"], tau_P=p["tau_P"][1])


def twin(runs, steps, every, export_u_at=(), log=print, precisions=PRECISIONS):
    """Advance the same runs in every precision; returns per-precision
    observation histories and exported velocity fields."""
    out = {}
    for prec in precisions:
        t0 = time.perf_counter()
        b = lbmve.Batch(runs, prec)
        hist, uf = [], {}
        m0 = [o["mass"] for o in b.observe()]
        done = 0
        while done < steps:
            k = min(every, steps - done)
            b.step(k)
            done += k
            obs = b.observe()
            log(f"  {prec} step {done}: D {[round(o['D'], 6) for o in obs][:3]}")
            hist.append([dict(step=o["step"], D=o["D"], theta=o["theta_deg"], mass=o["mass"],
                              status=o["status"]) for o in obs])
            if done in export_u_at:
                uf[done] = [b.export("u", r) for r in range(len(runs))]
        b.close()
        out[prec] = dict(hist=hist, u=uf, mass0=m0, seconds=time.perf_counter() - t0)
        log(f"{prec}: {steps} steps of {len(runs)} runs in {out[prec]['seconds']:.1f} s")
    return out


def compare(tw, nruns):
    rows = []
    ref = tw["fp64"]
    for prec in [p for p in ("fp32", "fp16s") if p in tw]:
        cur = tw[prec]
        for r in range(nruns):
            errs = []
            for h64, hp in zip(ref["hist"], cur["hist"]):
                a, b = h64[r], hp[r]
                errs.append(dict(step=a["step"], D64=a["D"], dD=abs(b["D"] - a["D"]),
                                 dtheta=abs(b["theta"] - a["theta"]),
                                 mass_drift=[(b["mass"][s] - cur["mass0"][r][s]) / cur["mass0"][r][s]
                                             for s in (0, 1)],
                                 status=b["status"]))
            uerr = {}
            for step, fields in ref["u"].items():
                u64, up = fields[r], cur["u"][step][r]
                uerr[step] = float(np.sqrt(((up - u64) ** 2).sum() / (u64 ** 2).sum()))
            rows.append(dict(precision=prec, run=r, max_dD=max(e["dD"] for e in errs),
                             max_dtheta=max(e["dtheta"] for e in errs),
                             u_rel_l2=uerr, checkpoints=errs))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--c2-steps", type=int, default=20000)
    ap.add_argument("--c3-steps", type=int, default=50000)
    ap.add_argument("--c3-lambdas", default="0.5,2")
    ap.add_argument("--skip-c2", action="store_true")
    ap.add_argument("--resume", default=None,
                    help="earlier report of the same sources: keep its parts, run the missing ones")
    ap.add_argument("--precisions", default=",".join(PRECISIONS),
                    help="comma-separated subset (fp64 is always included)")
    args = ap.parse_args(argv)
    precs = tuple(dict.fromkeys(["fp64"] + args.precisions.split(",")))
    log = lambda s: print(s, flush=True)
    from .build import source_hash
    report = {"source_hash": source_hash()}
    if args.resume:
        with open(args.resume) as fh:
            prev = json.load(fh)
        if prev.get("source_hash") != report["source_hash"]:
            raise SystemExit(f"{args.resume} was measured on other sources")
        report = prev
    if not args.skip_c2 and "c2" not in report:
        runs, tags = c2_runs()
        tw = twin(runs, args.c2_steps, 2000, export_u_at=(args.c2_steps,), log=log, precisions=precs)
        report["c2"] = dict(runs=tags, steps=args.c2_steps, compare=compare(tw, len(runs)),
                            seconds={p: tw[p]["seconds"] for p in precs})
        for row in report["c2"]["compare"]:
            log(f"c2 {row['precision']} run {row['run']}: max|dD| {row['max_dD']:.2e} "
                f"max|dtheta| {row['max_dtheta']:.2e} u rel L2 {row['u_rel_l2']}")
    report.setdefault("c3", [])
    done = {(r.get("lambda"), r["steps"]) for r in report["c3"]}
    ck = tuple(range(10000, args.c3_steps + 1, 10000)) or (args.c3_steps,)
    for lam in (float(v) for v in args.c3_lambdas.split(",") if v):
        if (lam, args.c3_steps) in done:
            continue
        p3, tag3 = c3_run(lam)
        tw3 = twin([p3], args.c3_steps, 2000, export_u_at=ck, log=log, precisions=precs)
        rep = dict(run=tag3, **{"lambda": lam}, steps=args.c3_steps, compare=compare(tw3, 1),
                   seconds={p: tw3[p]["seconds"] for p in precs})
        report["c3"].append(rep)
        for row in rep["compare"]:
            log(f"c3 lambda {lam} {row['precision']}: max|dD| {row['max_dD']:.2e} "
                f"max|dtheta| {row['max_dtheta']:.2e} u rel L2 {row['u_rel_l2']}")
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
