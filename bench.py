"""Throughput of the hybrid LB / FENE-P step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]

Workload: the matrix-viscoelastic droplet in confined shear on a 512x256x128
lattice (W = 128), droplet R = 32 (2R/W = 0.5) at mid-gap, FENE-P in the
matrix (L^2 = 400, De = 1, polymer fraction 0.4), viscosity ratio 0.5,
Ca = 0.25; synthetic initial state (sphere at rest, C = I), inputs resident
in HBM before the timed region.  One step = force pass + collide/stream/
FENE-P pass over every node.  Prints ONE JSON line.

The timed region replays the library's HIP graphs (the production path);
the per-pass durations for the roofline come from HIP events around each
pass in a second region of the same length on the same stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS (D3Q19x2 + FENE-P), % HBM roofline; Ca_cr sweeps/hour at +/-0.01"
# algorithmic bytes per lattice update: read and write every population of
# both components and every conformation component once
B_ALG = {"fp64": 2 * (38 + 6) * 8, "fp32": 2 * (38 + 6) * 4, "fp16s": 2 * (38 * 2 + 6 * 4)}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f16 storage / f32 compute"}


def workload_params(nx=512, ny=256, nz=128):
    from paper_1411_2181_amd import physics
    p, info = physics.lattice_params(nx, ny, nz, R=32.0, Ca=0.25, De=1.0, lam=0.5,
                                     phase="MV", L2=400.0, fraction=0.4, tau_matrix=1.0)
    return p, info


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1411_2181_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.startswith("lbm_"):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision):
    """HBM bytes per step from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_mv512.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    entry = t.get(precision)
    if not entry or entry.get("source_hash") != source_hash():
        return None
    return entry


def gpu_run(precision, steps, warmup, launch=None):
    import torch
    from paper_1411_2181_amd import lbmve
    p, info = workload_params()
    s = lbmve.Solver(p, precision)
    if launch:
        s.set_launch(**launch)
    nodes = p["nx"] * p["ny"] * p["nz"]
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_force, ms_update = s.step_profiled(steps)
    obs = s.observe()
    s.close()
    wall = t1 - t0
    return dict(nodes=nodes, wall=wall, ms_force=ms_force / steps, ms_update=ms_update / steps,
                obs=obs, params=p, info=info)


def cpu_baseline(seconds=12.0):
    """The FP64 oracle on a bounded sample of the same workload: the same
    physics on a 96x72x128 sub-box (full gap, R = 32 droplet), timed on one
    host core (the oracle is single-threaded NumPy)."""
    import numpy as np  # noqa: F401
    from oracle.solver import Oracle
    p, _ = workload_params(nx=96, ny=72, nz=128)
    o = Oracle(p)
    o.step(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    nodes = p["nx"] * p["ny"] * p["nz"]
    return dict(value=nodes * n / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"FP64 NumPy oracle, same parameters on a 96x72x128 sub-box "
                       f"({nodes} nodes, R=32), {n} steps after 1 warm-up step, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16s"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variants", default="fp16s", help="extra storage precisions to report")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                                   "multi-GPU slab decomposition is a design note"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)

    r = gpu_run(args.precision, args.steps, args.warmup)
    nodes, wall = r["nodes"], r["wall"]
    mlups = nodes * args.steps / wall / 1e6
    step_ms = r["ms_force"] + r["ms_update"]
    balg = B_ALG[args.precision]
    achieved = balg * nodes / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.precision)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "matrix-viscoelastic droplet in confined shear, 512x256x128 (W=128), "
                        "R=32, FENE-P in matrix L2=400 De=1 fraction 0.4, lambda=0.5, Ca=0.25",
            "nodes": nodes,
            "storage": args.precision,
            "u_wall": round(r["params"]["u_wall"], 6),
            "tau": [round(t, 5) for t in r["params"]["tau"]],
            "tau_P": round(r["params"]["tau_P"][1], 2),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step = k_force + k_update",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes_per_step"] if traffic else None,
            "bytes_alg_per_update": balg,
            "ms_force": round(r["ms_force"], 4),
            "ms_update": round(r["ms_update"], 4),
        },
    }
    variants = [v for v in args.variants.split(",") if v and v != args.precision]
    for v in variants:
        rv = gpu_run(v, args.steps, args.warmup)
        mv = rv["nodes"] * args.steps / rv["wall"] / 1e6
        sm = rv["ms_force"] + rv["ms_update"]
        ach = B_ALG[v] * rv["nodes"] / (sm * 1e-3) / 1e9
        out[f"variant_{v}"] = {"value": round(mv, 1), "unit": "MLUPS",
                               "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                               "ms_force": round(rv["ms_force"], 4),
                               "ms_update": round(rv["ms_update"], 4)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
