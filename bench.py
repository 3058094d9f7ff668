"""Throughput of the hybrid LB / FENE-P step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32] [--box 512x256x128]

Workload: the matrix-viscoelastic droplet in confined shear on a 512x256x128
lattice (W = 128), droplet R = 32 (2R/W = 0.5) at mid-gap, FENE-P in the
matrix (L^2 = 400, De = 1, polymer fraction 0.4), viscosity ratio 0.5, wall
speed 0.1 (Ca = 0.176 at the calibrated surface tension; the work per update
does not depend on Ca); synthetic
initial state (sphere at rest, C = I), inputs resident in HBM before the
timed region.  One step = one launch of the step kernel (forces, collision
and streaming of both components, FENE-P update) over every node.  Prints
ONE JSON line.

The launch shape is picked by the autotuner before the timed region (or
pinned with --launch).  After the warm-up steps, one untimed pass of K steps
instantiates every HIP-graph chunk that a K-step call replays; then five
regions of K steps each are timed (synchronised on both sides) and the
median region is reported.  The timed regions replay the library's HIP
graphs (the production path); the kernel duration for the roofline comes
from HIP events around each step kernel in a further region of the same
length on the same stream.  The step kernel is the whole step, so its
roofline is the step's; measured HBM traffic per dispatch comes from the
committed rocprofv3 counter summary (profiles/traffic_mv512.json) while the
kernel sources are unchanged.  A 1 GiB device-to-device copy timed in the
same process gives the measured bandwidth ceiling beside the 8 TB/s peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BOX = (512, 256, 128)
METRIC = "MLUPS (D3Q19x2 + FENE-P), % HBM roofline; Ca_cr sweeps/hour at +/-0.01"
# algorithmic bytes per lattice update: read and write every population of
# both components and every conformation component once
B_ALG = {"fp64": 2 * (38 + 6) * 8, "fp32": 2 * (38 + 6) * 4, "fp16s": 2 * (38 * 2 + 6 * 4)}
# bytes the step kernel must move per update: the algorithmic bytes plus the
# node densities and momenta (8 values, read and written) that carry the
# moments between steps
B_KERNEL = {"fp64": B_ALG["fp64"] + 2 * 8 * 8, "fp32": B_ALG["fp32"] + 2 * 8 * 4,
            "fp16s": B_ALG["fp16s"] + 2 * 8 * 4}
REGIONS = 5     # timed regions of K steps; the median is reported
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f16 storage / f32 compute"}


def workload_params(nx=512, ny=256, nz=128, u_wall=0.1):
    """Lattice parameters of the 512x256x128 matrix-viscoelastic case.

    Matrix solvent tau = 1.5 (the upper end of the window where the droplet
    interface is Laplace-consistent), lambda = 0.5 (tau_A = 4/3), De = 1,
    L^2 = 400, polymer fraction 0.4.  Ca = 0.25 would need U_w ~ 0.21 at the
    calibrated sigma; the wall speed is held at 0.1 instead (Ca = 0.176).  The
    work per lattice update does not depend on Ca."""
    from paper_1411_2181_amd import physics
    R, lam, frac = 32.0, 0.5, 0.4
    eta_B = physics.eta_of_tau(1.5)
    eta_M = eta_B / (1.0 - frac)
    tau_A = physics.tau_of_eta(lam * eta_M)
    sigma = physics.sigma_for(tau_A, 1.5)
    ca = min(0.25, u_wall * 2.0 * eta_M * R / (sigma * nz))
    p, info = physics.lattice_params(nx, ny, nz, R=R, Ca=ca, De=1.0, lam=lam, phase="MV",
                                     L2=400.0, fraction=frac, tau_matrix=1.5,
                                     u_max=u_wall * 1.0000001)
    info["Ca"] = ca
    return p, info


def measured_traffic(precision, launch, box=BOX):
    """HBM bytes per dispatch of each step kernel at this launch shape, from
    the committed rocprofv3 counter summary, if it was taken on the current
    kernel sources and the same lattice (else None)."""
    from paper_1411_2181_amd.build import source_hash
    path = os.path.join(ROOT, "profiles", "traffic_mv512.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    entry = t.get(precision)
    if not entry or entry.get("source_hash") != source_hash():
        return None
    if tuple(entry.get("box", BOX)) != tuple(box):
        return None
    # a persistent grid over the same tiles is taken to move the same bytes;
    # bz = 0 (whole columns) is the same tile table as bz = nz
    bz = launch["bz"] if launch["bz"] > 0 else box[2]
    return entry["launches"].get(f"{launch['bx']}x{launch['by']}x{bz}")


def gpu_run(precision, steps, warmup, launch=None, box=BOX, tau_minus=None):
    """Autotune (unless ``launch`` pins the shape), then the graph-replayed
    timed region, then ``steps`` eager steps with HIP events per pass.
    ``tau_minus`` switches the collision to two relaxation times."""
    import torch
    from paper_1411_2181_amd import autotune, lbmve
    p, info = workload_params(*box)
    if tau_minus:
        p["tau_minus"] = tuple(tau_minus)
    s = lbmve.Solver(p, precision)
    if launch:
        s.set_launch(**launch)
        tuned = None
    else:
        tuned = autotune.tune(s, steps=3, use_cache=False, save=False)
    nodes = p["nx"] * p["ny"] * p["nz"]
    s.step(warmup)
    # every graph chunk a K-step call replays is instantiated here, untimed
    s.step(steps)
    torch.cuda.synchronize()
    regions = []
    for _ in range(REGIONS):
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        regions.append(time.perf_counter() - t0)
    ms = s.step_profiled(steps) / steps
    obs = s.observe()
    launch = s.launch
    s.close()
    wall = sorted(regions)[len(regions) // 2]
    return dict(nodes=nodes, wall=wall, regions=regions, ms=ms, obs=obs, params=p,
                info=info, launch=launch, tuned=tuned, box=tuple(box), trt=bool(tau_minus))


def copy_bandwidth(gib=1, reps=5):
    """Measured ceiling for comparison: a device-to-device copy of ``gib`` GiB
    (read + written), timed with HIP events on the current stream; GB/s."""
    import torch
    n = (gib << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * (gib << 30) / (ms * 1e-3) / 1e9


def pmc_pass(precision, steps=4, launch=None):
    """Short run for hardware-counter collection: a 1 GiB device-to-device copy
    (the reference of known size for scaling FETCH_SIZE / WRITE_SIZE), then a
    few eager steps of the workload with every pass as its own dispatch (after
    the autotuner's candidates, unless ``launch`` pins the shape)."""
    import torch
    from paper_1411_2181_amd import autotune, lbmve
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    flush = torch.empty_like(a)
    flush.fill_(2.0)       # evict a from the last-level cache
    b.copy_(a)             # 1 GiB read + 1 GiB written
    torch.cuda.synchronize()
    del a, b, flush
    p, _ = workload_params()
    s = lbmve.Solver(p, precision)
    if launch:
        s.set_launch(**launch)
    else:
        # non-persistent candidates only: their grids identify (bx, by, bz)
        autotune.tune(s, steps=2, use_cache=False, save=False, persistent=False)
    s.step_profiled(steps)
    s.close()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline_child(seconds):
    """Runs in a child process pinned to one core, thread pools at 1."""
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
    import threading
    return dict(value=nodes * n / dt / 1e6, n=n, dt=dt, nodes=nodes,
                threads=threading.active_count(),
                affinity=sorted(os.sched_getaffinity(0)))


def cpu_baseline(seconds=12.0):
    """The FP64 oracle on a bounded sample of the same workload: the same
    physics on a 96x72x128 sub-box (full gap, R = 32 droplet), in a child
    process pinned to one host core with every thread pool at one thread
    (the oracle is single-threaded NumPy)."""
    import subprocess
    core = min(os.sched_getaffinity(0))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1", NUMEXPR_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    code = ("import os, sys, json; os.sched_setaffinity(0, {%d}); sys.path.insert(0, %r); "
            "import bench; print(json.dumps(bench._cpu_baseline_child(%r)))"
            % (core, ROOT, seconds))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline failed: {r.stderr[-2000:]}")
    c = json.loads(r.stdout.strip().splitlines()[-1])
    return dict(value=c["value"], unit="MLUPS", cores=len(c["affinity"]), kind="oracle",
                cpu=_cpu_model(), threads_env=1,
                sample=f"FP64 NumPy oracle, same parameters on a 96x72x128 sub-box "
                       f"({c['nodes']} nodes, R=32), {c['n']} steps after 1 warm-up step, "
                       f"{c['dt']:.1f} s, one process pinned to core {c['affinity'][0]}")


def roofline(precision, r):
    """Roofline of the step kernel (the whole step in one launch) from its
    HIP-event duration: algorithmic bytes per update (every population and
    C component read and written once) over the kernel time."""
    nodes = r["nodes"]
    ms = r["ms"]
    balg = B_ALG[precision]
    ach = balg * nodes / (ms * 1e-3) / 1e9
    # the committed counters are of the BGK kernel
    tr = None if r.get("trt") else measured_traffic(precision, r["launch"], r.get("box", BOX))
    out = {
        "bound": "hbm",
        "kernel": "k_step (forces, collide-stream of both components, FENE-P: the whole step)",
        "achieved": round(ach, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": tr["k_step"]["bytes"] if tr else None,
        "bytes_alg_per_node": balg,
        "bytes_min_per_node": B_KERNEL[precision],
        "ms_per_launch": round(ms, 4),
        "traffic_per_node": tr["k_step"]["bytes_per_node"] if tr else None,
    }
    if tr:
        out["achieved_actual"] = round(tr["k_step"]["bytes"] / (ms * 1e-3) / 1e9, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16s"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variants", default="fp16s", help="extra storage precisions to report")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="short run for rocprofv3 counter collection (prints no JSON)")
    ap.add_argument("--launch", default="",
                    help="pin the launch shape BXxBYxBZ[xP] instead of autotuning (profiling runs)")
    ap.add_argument("--box", default="512x256x128",
                    help="lattice NXxNYxNZ (default: the full case; 64x256x128 is one GPU's "
                         "x-slab of it in an 8-way decomposition)")
    ap.add_argument("--tau-minus", default="",
                    help="A,B: odd-moment relaxation times (two-relaxation-time collision "
                         "instead of BGK; the throughput of that variant)")
    args = ap.parse_args()
    box = tuple(int(t) for t in args.box.lower().split("x"))
    tau_minus = tuple(float(t) for t in args.tau_minus.split(",")) if args.tau_minus else None
    launch = None
    if args.launch:
        v = [int(t) for t in args.launch.lower().split("x")]
        launch = dict(bx=v[0], by=v[1], bz=v[2], persistent=v[3] if len(v) > 3 else 0)
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU only; "
                                   "multi-GPU slab decomposition is a design note"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.pmc_pass:
        pmc_pass(args.precision, launch=launch)
        return

    r = gpu_run(args.precision, args.steps, args.warmup, launch, box, tau_minus)
    nodes, wall = r["nodes"], r["wall"]
    mlups = nodes * args.steps / wall / 1e6
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "timed_regions": {"count": REGIONS, "reported": "median",
                          "ms_per_step": [round(t / args.steps * 1e3, 4) for t in r["regions"]]},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "matrix-viscoelastic droplet in confined shear, "
                        f"{box[0]}x{box[1]}x{box[2]} (W={box[2]}), "
                        "R=32, FENE-P in matrix L2=400 De=1 fraction 0.4, lambda=0.5, "
                        f"Ca={r['info']['Ca']:.3f} (U_w=0.1)",
            "nodes": nodes,
            "storage": args.precision,
            "u_wall": round(r["params"]["u_wall"], 6),
            "tau": [round(t, 5) for t in r["params"]["tau"]],
            "tau_P": round(r["params"]["tau_P"][1], 2),
            "launch": r["launch"],
            "collision": f"TRT tau_minus={list(tau_minus)}" if tau_minus else "BGK",
        },
        "roofline": roofline(args.precision, r),
    }
    variants = [v for v in args.variants.split(",") if v and v != args.precision]
    for v in variants:
        rv = gpu_run(v, args.steps, args.warmup, box=box, tau_minus=tau_minus)
        mv = rv["nodes"] * args.steps / rv["wall"] / 1e6
        out[f"variant_{v}"] = {"value": round(mv, 1), "unit": "MLUPS",
                               "ms_per_step": round(rv["wall"] / args.steps * 1e3, 4),
                               "launch": rv["launch"], "roofline": roofline(v, rv)}
    out["roofline"]["copy_ceiling"] = {
        "what": "1 GiB device-to-device copy (read + written), HIP events",
        "GBs": round(copy_bandwidth(), 1)}
    out["roofline"]["copy_ceiling"]["frac"] = round(out["roofline"]["copy_ceiling"]["GBs"] /
                                                    HBM_PEAK_GBS, 4)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
