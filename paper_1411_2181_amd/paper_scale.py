"""Critical capillary number at the paper's dimensionless set-up (host driver).

Section 3 of the paper brackets Ca_cr for Newtonian, droplet-viscoelastic
and matrix-viscoelastic droplets at confinement 2R/W = 0.52 and 0.7, De = 2,
viscosity ratio 1 and Reynolds number about 0.5, in boxes about
20.5R x 2.56R x W (its Figs. 2-3).  With BGK and the velocity-shift forcing
the Shan-Chen droplet stays Laplace-consistent only for tau of about 1-1.5,
which caps the matrix viscosity and hence the Ca reachable at a safe wall
speed below every printed Ca_cr.  The two-relaxation-time collision
separates the two roles of tau: the odd-moment time tau^- (which carries the
momentum and so the velocity shift) is held at one value for both
components, where the interface is well behaved, while the even-moment time
tau^+ sets each component's viscosity freely.

Stages, all on the GPU through the batched solver:
  1. sigma by the Laplace law for each mode's (tau^+_A, tau^+_B, tau^-)
     (static droplets of R = 10, 12, 14 in 48^3 boxes, as in calibrate.py);
  2. every (mode, Ca) run in one batch, up to t_end = T_TEM tau_em steps
     (the paper's last snapshot is at t/tau_em = 100), checked for break-up
     every --every steps by connected-component labelling; a broken run is
     masked at once;
  3. per mode, two brackets with the Reynolds number at each: by break-up
     ([largest Ca that stayed whole below the smallest that broke, that
     smallest]) and by the shape criterion of the paper's figures, which
     tell sub-critical droplets (a steady shape) from super-critical ones
     (still stretching, or broken): a run is steady when its length L_p
     changed by less than STEADY_TOL over its last STEADY_TEM tau_em.

    python -m paper_1411_2181_amd.paper_scale OUT.json --R 32 --c 0.52 --tau-plus 6 \\
        --tau-minus 1 --De 2 --N 0.28,0.32,0.36 --DV 0.36,0.4 --MV 0.28,0.32
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import calibrate, lbmve, physics, sweep

RHO_REF = physics.RHO_MAJOR + physics.RHO_MINOR
# box of the paper's runs in units of R: 1024 x 128 x W at R = 50
BOX_X, BOX_Y = 1024.0 / 50.0, 128.0 / 50.0
T_TEM = 100.0
STEADY_TEM, STEADY_TOL = 10.0, 0.02


def eta_of(tau_plus: float) -> float:
    return RHO_REF * (tau_plus - 0.5) / 3.0


def tau_of(eta: float) -> float:
    return 0.5 + 3.0 * eta / RHO_REF


def viscosities(mode: str, eta_M: float, lam: float, fraction: float):
    """(tau^+_A, tau^+_B, eta_P of A, eta_P of B) with lambda on the total
    viscosities (Section 3): N, DV (polymer in the droplet) or MV."""
    if mode == "N":
        return tau_of(lam * eta_M), tau_of(eta_M), 0.0, 0.0
    if mode == "DV":
        eta_d = lam * eta_M
        return tau_of((1.0 - fraction) * eta_d), tau_of(eta_M), fraction * eta_d, 0.0
    if mode == "MV":
        return tau_of(lam * eta_M), tau_of((1.0 - fraction) * eta_M), 0.0, fraction * eta_M
    raise ValueError(mode)


def sigma_runs(taus, tau_minus: float, G: float):
    runs = []
    for ta, tb in taus:
        for R in calibrate.RADII:
            d = calibrate._run_params(ta, tb, R, G=G)
            d["tau_minus"] = (tau_minus, tau_minus)
            runs.append(d)
    return runs


def measure_sigma(taus, tau_minus: float, G: float, precision: str, steps: int, log=print,
                  densities=None):
    """sigma (least squares of dp = 2 sigma / R_eff over the three radii) and
    the largest relative residual, per (tau^+_A, tau^+_B) pair (tau_minus = 0:
    BGK).  ``densities`` (a list) receives the component densities at the
    centre and in the far matrix of the middle radius's droplet."""
    runs = sigma_runs(taus, tau_minus, G)
    b = lbmve.Batch(runs, precision)
    b.step([steps] * len(runs))
    out = []
    nr = len(calibrate.RADII)
    for k, pair in enumerate(taus):
        x, y = [], []
        for j in range(nr):
            rho = b.export("rho", k * nr + j)
            dp, reff = calibrate.laplace_measure(rho, G)
            x.append(1.0 / reff)
            y.append(dp)
            if densities is not None and j == nr // 2:
                c = calibrate.BOX // 2
                densities.append(dict(A_in=float(rho[0][c, c, c]), B_in=float(rho[1][c, c, c]),
                                      A_out=float(rho[0][c, 1, 1]), B_out=float(rho[1][c, 1, 1])))
        x, y = np.array(x), np.array(y)
        sig = float(x @ y / (x @ x) / 2.0)
        resid = float(np.abs(y - 2.0 * sig * x).max() / np.abs(y).max())
        out.append((sig, resid))
        log(f"sigma at tau+ = {pair}, tau- = {tau_minus}: {sig:.5f} (Laplace residual {resid:.2%})")
    b.close()
    return out


def run_params(mode, Ca, R, c, De, lam, fraction, L2, eta_M, tau_minus, sigma, G, u_max,
               box_x=BOX_X):
    W = int(round(2.0 * R / c))
    nx, ny = int(round(box_x * R)), int(round(BOX_Y * R))
    ta, tb, ePA, ePB = viscosities(mode, eta_M, lam, fraction)
    gdot = Ca * sigma / (eta_M * R)
    u_wall = gdot * W / 2.0
    if u_wall > u_max:
        raise ValueError(f"{mode} Ca={Ca}: U_w = {u_wall:.3f} exceeds {u_max}")
    tau_P = De / gdot if mode != "N" else 1.0
    p = dict(nx=nx, ny=ny, nz=W, u_wall=u_wall, radius=float(R), cx=-1.0, cy=-1.0, cz=-1.0,
             rho_major=physics.RHO_MAJOR, rho_minor=physics.RHO_MINOR, G=G,
             tau=(ta, tb), tau_minus=(tau_minus, tau_minus), tau_P=(tau_P, tau_P),
             eta_P=(ePA, ePB), L2=(L2, L2), chi_lo=0.0, chi_hi=0.0)
    info = dict(sigma=sigma, gamma_dot=gdot, eta_M=eta_M, tau_em=R * eta_M / sigma,
                Re=physics.RHO_MAJOR * gdot * R * R / eta_M, W=W, box=[nx, ny, W])
    return p, info


def bracket(rows, key="broken"):
    """[largest Ca below the smallest Ca with row[key] true among the runs
    with it false (status 0), that Ca] (None where no run of that kind
    exists)."""
    hit = sorted(r["Ca"] for r in rows if r[key])
    hi = hit[0] if hit else None
    miss = [r["Ca"] for r in rows if not r[key] and r["status"] == 0
            and (hi is None or r["Ca"] < hi)]
    lo = max(miss) if miss else None
    return lo, hi


def steady(history, tau_em: float, window_tem: float = STEADY_TEM, tol: float = STEADY_TOL) -> bool:
    """L_p at the last check within tol (relative) of L_p at the last check
    at least window_tem tau_em earlier."""
    if not history:
        return False
    t1, lp1 = history[-1]["step"], history[-1]["Lp_over_2R"]
    earlier = [h for h in history if h["step"] <= t1 - window_tem * tau_em]
    if not earlier:
        return False
    lp0 = earlier[-1]["Lp_over_2R"]
    return abs(lp1 - lp0) <= tol * lp0


def brackets_of(rows, modes):
    """Per mode: the break-up bracket and the shape bracket (super-critical =
    broken or still stretching), each with Re at its ends."""
    out = {}
    for mode in modes:
        rs = [dict(r, supercritical=r["broken"] or not r["steady"]) for r in rows if r["mode"] == mode]
        entry = {}
        for name, key in (("breakup", "broken"), ("shape", "supercritical")):
            lo, hi = bracket(rs, key)
            re_at = [r["Re"] for r in rs if r["Ca"] in (lo, hi)]
            entry[name] = dict(Ca_cr_lo=lo, Ca_cr_hi=hi, Re=[min(re_at), max(re_at)] if re_at else None)
        out[mode] = entry
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("out")
    ap.add_argument("--R", type=float, default=32.0)
    ap.add_argument("--c", type=float, default=0.52, help="confinement 2R/W")
    ap.add_argument("--tau-plus", type=float, default=6.0, help="even-moment tau of the matrix (total viscosity)")
    ap.add_argument("--tau-minus", type=float, default=1.0, help="odd-moment tau of both components")
    ap.add_argument("--G", type=float, default=physics.G_DEFAULT)
    ap.add_argument("--De", type=float, default=2.0)
    ap.add_argument("--lam", type=float, default=1.0)
    ap.add_argument("--fraction", type=float, default=0.4)
    ap.add_argument("--L2", type=float, default=100.0)
    ap.add_argument("--N", default="", help="Ca list of the Newtonian droplet")
    ap.add_argument("--DV", default="", help="Ca list, polymer in the droplet")
    ap.add_argument("--MV", default="", help="Ca list, polymer in the matrix")
    ap.add_argument("--t-tem", type=float, default=T_TEM, help="run length in tau_em")
    ap.add_argument("--box-x", type=float, default=BOX_X, help="box length in units of R")
    ap.add_argument("--every", type=int, default=2000)
    ap.add_argument("--u-max", type=float, default=0.19)
    ap.add_argument("--sigma-steps", type=int, default=calibrate.STEPS)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16s"])
    ap.add_argument("--combine", default="",
                    help="A.json,B.json: merge the rows of earlier scans (same set-up) into OUT")
    ap.add_argument("--window", default="",
                    help="'tA,tB;tA,tB;...': only the static-droplet stage, for these tau^+ pairs, "
                         "with BGK (tau = tau^+) and with --tau-minus")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.window:
        pairs = [tuple(float(v) for v in p.split(",")) for p in args.window.split(";")]
        res = {}
        for name, tm in (("bgk", 0.0), (f"trt tau_minus={args.tau_minus}", args.tau_minus)):
            dens = []
            sig = measure_sigma(pairs, tm, args.G, args.precision, args.sigma_steps, log, dens)
            res[name] = [dict(tau_plus=list(p), sigma=s, laplace_residual=r, densities_R12=d)
                         for p, (s, r), d in zip(pairs, sig, dens)]
        with open(args.out, "w") as fh:
            json.dump(dict(G=args.G, steps=args.sigma_steps, radii=list(calibrate.RADII),
                           box=calibrate.BOX, precision=args.precision, window=res), fh, indent=1)
        return 0

    if args.combine:
        scans = [json.load(open(p)) for p in args.combine.split(",")]
        rows = sorted((r for s in scans for r in s["rows"]), key=lambda r: (r["mode"], r["Ca"]))
        modes = [m for m in ("N", "DV", "MV") if any(r["mode"] == m for r in rows)]
        out = {k: v for k, v in scans[0].items() if k not in ("rows", "brackets", "seconds", "seconds_runs")}
        out.update(scans=args.combine.split(","), brackets=brackets_of(rows, modes),
                   sigma={m: [s["sigma"][m] for s in scans if m in s.get("sigma", {})] for m in modes},
                   rows=rows)
        for m in modes:
            log(f"{m}: {out['brackets'][m]}")
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1, default=float)
        return 0

    t0 = time.perf_counter()
    eta_M = eta_of(args.tau_plus)
    modes = [(m, [float(v) for v in getattr(args, m).split(",") if v]) for m in ("N", "DV", "MV")]
    modes = [(m, cas) for m, cas in modes if cas]
    taus = [viscosities(m, eta_M, args.lam, args.fraction)[:2] for m, _ in modes]
    sig = measure_sigma(taus, args.tau_minus, args.G, args.precision, args.sigma_steps, log)
    specs, prepared, tags = [], [], []
    for (mode, cas), (sigma, _res) in zip(modes, sig):
        for ca in cas:
            p, info = run_params(mode, ca, args.R, args.c, args.De, args.lam, args.fraction,
                                 args.L2, eta_M, args.tau_minus, sigma, args.G, args.u_max,
                                 box_x=args.box_x)
            specs.append(sweep.RunSpec(args.R, args.c, ca, args.De if mode != "N" else 0.0,
                                       args.lam, args.L2, args.fraction, phase=mode))
            prepared.append((p, info))
            tags.append(dict(mode=mode, Ca=ca))
    t_end = int(round(args.t_tem * prepared[0][1]["tau_em"]))
    nodes = sum(p["nx"] * p["ny"] * p["nz"] for p, _ in prepared)
    log(f"{len(specs)} runs, {nodes / 1e6:.1f} M nodes, up to {t_end} steps "
        f"(tau_em {prepared[0][1]['tau_em']:.0f}, Re at the first Ca {prepared[0][1]['Re']:.2f})")
    res, sec = sweep.simulate(specs, args.precision, t_end=t_end, every=args.every,
                              progress=log, prepared=prepared)
    rows = []
    for t, r in zip(tags, res):
        tem = r.info["tau_em"]
        hist = [dict(step=h[0], t_over_tau_em=h[0] / tem, D=h[1], theta=h[2],
                     Lp_over_2R=h[3] / (2 * args.R), pieces=h[4],
                     volume_over_initial=h[5] / (4.0 / 3.0 * math.pi * args.R ** 3))
                for h in r.history]
        rows.append(dict(t, tau_plus=list(r.params["tau"]), tau_minus=args.tau_minus,
                         steady=steady(hist, tem),
                         u_wall=r.params["u_wall"], tau_P=r.params["tau_P"][0], Re=r.info["Re"],
                         tau_em=tem, broken=r.broken, step_break=r.step_break, status=r.status,
                         steps=r.steps, t_break_over_tau_em=(r.step_break / tem) if r.broken else None,
                         daughter_nodes=r.pieces, Lp_max_over_2R=max(h["Lp_over_2R"] for h in hist),
                         history=hist))
        log(f"{t['mode']:2s} Ca={t['Ca']:.3f} Re={r.info['Re']:.2f}: "
            + (f"breaks at t/tau_em = {r.step_break / tem:.1f} into {len(r.pieces)} {r.pieces}"
               if r.broken else f"whole after {r.steps} steps (status {r.status})")
            + f", max Lp/2R {rows[-1]['Lp_max_over_2R']:.2f}")
    brackets = brackets_of(rows, [m for m, _ in modes])
    sigmas = {m: dict(sigma=s, laplace_residual=res) for (m, _), (s, res) in zip(modes, sig)}
    for m, _ in modes:
        log(f"{m}: {brackets[m]}")
    out = dict(R=args.R, c=args.c, tau_plus_matrix=args.tau_plus, tau_minus=args.tau_minus,
               eta_M=eta_M, G=args.G, De=args.De, lam=args.lam, fraction=args.fraction, L2=args.L2,
               precision=args.precision, t_over_tau_em=args.t_tem, t_end=t_end, every=args.every,
               box=prepared[0][1]["box"], nodes_total=nodes, seconds=time.perf_counter() - t0,
               seconds_runs=sec, sigma=sigmas, brackets=brackets, rows=rows)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1, default=float)
    return 0


if __name__ == "__main__":
    sys.exit(main())
