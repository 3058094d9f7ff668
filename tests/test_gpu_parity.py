"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar (FP64): per exported field max|GPU - oracle| / max|oracle| <= 1e-10 after
2000 steps of the 32^3 droplet cases, and <= 1e-12 after 10 steps from random
states on ragged lattices; observables relative <= 1e-10 (orientation
absolute <= 1e-8 degrees).  Integer results (component counts) bit-exact.
Bit-identity where the arithmetic is the same: launch shapes, batches,
repeated runs and checkpoint/restart.
"""
import math

import numpy as np
import pytest

import workloads as WL
from oracle import d3q19
from oracle.components import component_sizes
from oracle.observables import observe
from oracle.solver import Oracle
from tests import oracle_pool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2181_amd import lbmve
    lbmve.lib()
    return lbmve


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _fields(s):
    return dict(f=s.export("f"), C=s.export("C"), rho=s.export("rho"), u=s.export("u"))


def _check_obs(g, o, tol=1e-10):
    assert abs(g["mass"][0] - o["mass"][0]) <= tol * abs(o["mass"][0])
    assert abs(g["mass"][1] - o["mass"][1]) <= tol * abs(o["mass"][1])
    assert abs(g["D"] - o["D"]) <= tol * max(abs(o["D"]), 1e-6)
    assert abs(g["theta_deg"] - o["theta_deg"]) <= 1e-8 or abs(o["D"]) < 1e-6
    for a in range(3):
        assert abs(g["centroid"][a] - o["centroid"][a]) <= tol * 100
    assert g["Lp"] == o["Lp"]
    assert abs(g["trC_max"] - o["trC_max"]) <= tol * o["trC_max"]
    if "umax" in o:
        assert abs(g["umax"] - o["umax"]) <= tol * max(o["umax"], 1e-12)


def test_init_state_exact(lbm):
    d = WL.small_droplet_viscoelastic()
    s = lbm.Solver(d, "fp64")
    o = Oracle(d)
    assert np.array_equal(s.export("f"), o.f)
    assert np.array_equal(s.export("C"), o.C)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_init_state_with_seeded_noise(lbm, precision):
    """The optional initial density noise (seed, relative amplitude 1 %) is
    the oracle's, word for word of the counter-based generator: FP64 fields
    bit-exact, FP32 to its rounding; 100 steps later still at the bar."""
    d = dict(WL.small_droplet_viscoelastic(), seed=987654321, init_noise=0.01)
    s = lbm.Solver(d, precision)
    o = Oracle(d)
    rho = s.export("rho")
    ref = np.stack([o.f[0].sum(axis=0), o.f[1].sum(axis=0)])
    print(f"case seeded noise {precision}: rho spread {rho[0].std():.2e}", flush=True)
    # (ref sums the populations, so it carries their rounding: 1e-15)
    if precision == "fp64":
        assert np.array_equal(s.export("f"), o.f) and rel(rho, ref) <= 1e-15
    else:
        assert rel(rho, ref) <= 1e-7
    # the noise is there, within its amplitude
    rel0 = np.abs(rho / np.stack([Oracle(dict(d, init_noise=0.0)).f[c].sum(axis=0)
                                  for c in (0, 1)]) - 1.0)
    assert 0.009 < rel0.max() <= 0.01 + 1e-6
    s.step(100)
    o.step(100)
    assert rel(s.export("f"), o.f) <= (1e-10 if precision == "fp64" else 1e-5)
    s.close()


@pytest.mark.parametrize("shape_xyz", [(17, 9, 12), (33, 5, 40)])
@pytest.mark.parametrize("visc", ["none", "A", "B"])
def test_random_state_ragged_parity(lbm, shape_xyz, visc):
    nx, ny, nz = shape_xyz
    eta = {"none": (0.0, 0.0), "A": (0.05, 0.0), "B": (0.0, 0.05)}[visc]
    d = WL.base_params(nx=nx, ny=ny, nz=nz, radius=3.0, u_wall=0.02, tau=(0.8, 1.3),
                       tau_P=(20.0, 30.0), eta_P=eta, L2=(60.0, 80.0))
    print(f"case ragged {shape_xyz} visc={visc}", flush=True)
    f0 = WL.random_populations((nz, ny, nx), d3q19.W, seed=7)
    C0 = WL.random_conformation((nz, ny, nx), seed=8)
    s = lbm.Solver(d, "fp64")
    s.import_("f", f0)
    s.import_("C", C0)
    s.step(10)
    g = _fields(s)
    o = Oracle(d, f=f0, C=C0)
    o.step(10)
    assert rel(g["f"], o.f) <= 1e-12
    assert rel(g["C"], o.C) <= 1e-12
    assert rel(g["rho"], o.density()) <= 1e-12
    assert rel(g["u"], o.velocity()) <= 1e-11
    go = s.observe()
    oo = observe(o.f, o.C, o.velocity())
    assert abs(go["mass"][0] - oo["mass"][0]) <= 1e-12 * oo["mass"][0]
    assert abs(go["trC_max"] - oo["trC_max"]) <= 1e-12 * oo["trC_max"]
    s.close()


CASES = {"newtonian": WL.small_newtonian, "droplet_visc": WL.small_droplet_viscoelastic,
         "matrix_visc": WL.small_matrix_viscoelastic}


@pytest.fixture(scope="module")
def oracle_2000():
    # start the three long oracle runs in worker processes right away
    return {k: oracle_pool.submit(fn(), 2000) for k, fn in CASES.items()}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", list(CASES))
def test_small_droplet_2000_steps_parity(lbm, oracle_2000, case):
    d = CASES[case]()
    print(f"case 32^3 {case} 2000 steps", flush=True)
    s = lbm.Solver(d, "fp64")
    s.step(2000)
    g = _fields(s)
    go = s.observe(components=True)
    o = oracle_2000[case].result()
    for k in ("f", "C", "rho", "u"):
        assert rel(g[k], o[k]) <= 1e-10, k
    _check_obs(go, o["obs"])
    assert go["status"] == 0 and o["status"] == 0
    assert go["n_components"] == 1
    # the droplet did deform under shear (the check is not trivial)
    assert go["D"] > 1e-3
    s.close()


def test_launch_shapes_bit_identical(lbm):
    d = WL.small_droplet_viscoelastic()
    ref = None
    for shape in [dict(bx=16, by=8, bz=1), dict(bx=8, by=16, bz=3),
                  dict(bx=16, by=8, bz=8, persistent=64), dict(bx=8, by=16, bz=32),
                  dict(bx=16, by=8, bz=5, persistent=8), dict(bx=16, by=8, bz=0)]:
        s = lbm.Solver(d, "fp64")
        s.set_launch(**shape)
        s.step(25)
        out = (s.export("f"), s.export("C"))
        s.close()
        if ref is None:
            ref = out
        else:
            df = float(np.abs(out[0] - ref[0]).max() / np.abs(ref[0]).max())
            dC = float(np.abs(out[1] - ref[1]).max() / np.abs(ref[1]).max())
            print(f"  {shape}: max rel diff f {df:.2e}, C {dC:.2e}", flush=True)
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), shape


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_grouped_addressing_bit_identical(lbm, precision):
    """The population arrays addressed in groups of four (the path of runs
    whose arrays span more than 4 GiB) give the same bits as one base, on a
    ragged lattice with walls and a polymer phase."""
    d = WL.base_params(nx=37, ny=21, nz=19, radius=6.0, u_wall=0.05, tau=(1.0, 0.8),
                       tau_P=(1.0, 5.0), eta_P=(0.0, 0.05), L2=(100.0, 100.0))
    print(f"case grouped addressing 37x21x19 {precision}", flush=True)
    out = []
    for grouped in (0, 1):
        s = lbm.Solver(d, precision)
        shape = dict(bx=16, by=8, bz=7) if precision == "fp64" else dict(bx=32, by=8, bz=7)
        s.set_launch(**shape, grouped=grouped)
        assert s.launch["grouped"] == grouped
        s.step(40)
        out.append((s.export("f"), s.export("C"), s.export("rho")))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_repeat_and_checkpoint_bit_identical(lbm, precision):
    d = WL.small_matrix_viscoelastic()
    a = lbm.Solver(d, precision)
    a.step(60)
    fa, Ca = a.export("f"), a.export("C")
    b = lbm.Solver(d, precision)
    b.step(60)
    assert np.array_equal(b.export("f"), fa) and np.array_equal(b.export("C"), Ca)
    # raw-state checkpoint at step 30, restart in a fresh context
    c = lbm.Solver(d, precision)
    c.step(30)
    blob = c.save_state()
    r = lbm.Solver(d, precision)
    r.load_state(blob)
    assert r.observe()["step"] == 30
    r.step(30)
    assert np.array_equal(r.export("f"), fa) and np.array_equal(r.export("C"), Ca)
    # restart from the exported FP64 fields: exact up to the re-encoding
    x = lbm.Solver(d, precision)
    x.import_("f", c.export("f"))
    x.import_("C", c.export("C"))
    x.step(30)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "fp16s": 1e-2}[precision]
    assert np.max(np.abs(x.export("f") - fa)) <= tol * np.max(np.abs(fa))
    for s in (a, b, c, r, x):
        s.close()


def test_state_of_a_batch_run_round_trips(lbm):
    """Raw state of one run of a batch restores bit for bit into the same run
    of a fresh batch; blobs of another box or precision are rejected."""
    runs = [WL.small_droplet_viscoelastic(),
            WL.base_params(nx=20, ny=24, nz=18, radius=5.0, tau=(1.0, 0.8),
                           tau_P=(1.0, 50.0), eta_P=(0.0, 0.05), u_wall=0.01),
            WL.base_params(nx=17, ny=9, nz=12, radius=3.0, u_wall=0.02)]
    for prec in ("fp32", "fp16s"):
        a = lbm.Batch(runs, prec)
        a.step([30, 17, 25])
        blob = a.save_state(1)
        b = lbm.Batch(runs, prec)
        b.step([3, 0, 0])
        b.load_state(blob, 1)
        assert b.observe()[1]["step"] == 17
        a.step([0, 11, 0])
        b.step([0, 11, 0])
        assert np.array_equal(a.export("f", 1), b.export("f", 1)), prec
        assert np.array_equal(a.export("C", 1), b.export("C", 1)), prec
        with pytest.raises(lbm.LbmError):
            b.load_state(blob, 2)          # another box
        with pytest.raises(lbm.LbmError):
            b.load_state(blob[:-1], 1)     # wrong size
        a.close()
        b.close()
    c = lbm.Batch(runs, "fp64")
    with pytest.raises(lbm.LbmError):
        c.load_state(blob, 1)              # FP16S blob into an FP64 context (size differs)
    c.close()


def test_batch_equals_single_runs(lbm):
    runs = [WL.small_droplet_viscoelastic(),
            WL.base_params(nx=20, ny=24, nz=18, radius=5.0, tau=(1.0, 0.8),
                           tau_P=(1.0, 50.0), eta_P=(0.0, 0.05), u_wall=0.01),
            WL.base_params(nx=17, ny=9, nz=12, radius=3.0, u_wall=0.02)]
    steps = [30, 17, 25]
    for prec in ("fp64", "fp32", "fp16s"):
        b = lbm.Batch(runs, prec)
        b.step(steps)
        for r, d in enumerate(runs):
            s = lbm.Solver(d, prec)
            s.step(steps[r])
            assert np.array_equal(b.export("f", r), s.export("f")), (prec, r)
            assert np.array_equal(b.export("C", r), s.export("C")), (prec, r)
            assert b.steps_done(r) == steps[r]
            s.close()
        obs = b.observe()
        assert [o["step"] for o in obs] == steps
        # runs given zero steps are masked: their state does not change
        before = [b.export("f", r) for r in range(len(runs))]
        b.step([0, 4, 0])
        assert [b.steps_done(r) for r in range(len(runs))] == [steps[0], steps[1] + 4, steps[2]]
        assert np.array_equal(b.export("f", 0), before[0])
        assert np.array_equal(b.export("f", 2), before[2])
        assert not np.array_equal(b.export("f", 1), before[1])
        b.step([0, 0, 0])
        assert np.array_equal(b.export("f", 0), before[0])
        b.close()


UNEVEN_BATCH = [
    WL.base_params(nx=20, ny=12, nz=16, radius=5.0, u_wall=0.01, tau=(0.8, 1.0),
                   tau_P=(50.0, 1.0), eta_P=(0.05, 0.0), L2=(100.0, 100.0)),
    WL.base_params(nx=17, ny=9, nz=12, radius=3.0, u_wall=0.02),
    WL.base_params(nx=24, ny=10, nz=14, radius=4.0, u_wall=0.015, tau=(1.0, 0.8),
                   tau_P=(1.0, 40.0), eta_P=(0.0, 0.04), L2=(100.0, 60.0)),
    WL.base_params(nx=13, ny=16, nz=20, radius=4.5, u_wall=-0.01, tau=(1.2, 0.9), G=0.8),
]
UNEVEN_STEPS = [300, 170, 250, 90]


@pytest.mark.timeout(600)
def test_uneven_batch_matches_oracle(lbm):
    """Four runs of different boxes, phases and parameters in one FP64
    batch, each given its own step count: every run's fields against the
    oracle (the batched tile table, per-run parameters and masking, tiles of
    each run's own height)."""
    futs = [oracle_pool.submit(d, n) for d, n in zip(UNEVEN_BATCH, UNEVEN_STEPS)]
    b = lbm.Batch(UNEVEN_BATCH, "fp64")
    # tiles spanning each run's whole height (different per run), taken in
    # turn by a persistent grid of 16 workgroups
    b.set_launch(bx=16, by=8, bz=0, persistent=16)
    b.step(UNEVEN_STEPS)
    obs = b.observe()
    for r, fut in enumerate(futs):
        o = fut.result()
        print(f"case uneven batch run {r}: {UNEVEN_STEPS[r]} steps", flush=True)
        assert obs[r]["step"] == UNEVEN_STEPS[r]
        for k, ref in (("f", o["f"]), ("C", o["C"]), ("rho", o["rho"]), ("u", o["u"])):
            assert rel(b.export(k, r), ref) <= 1e-10, (r, k)
        _check_obs(obs[r], o["obs"])
    b.close()


def test_nan_and_fene_flags(lbm):
    d = WL.small_droplet_viscoelastic()
    s = lbm.Solver(d, "fp64")
    s.step(3)
    assert s.observe()["status"] == 0
    f = s.export("f")
    f[0, 3, 10, 10, 10] = np.nan
    s.import_("f", f)
    s.step(2)
    assert s.observe()["status"] == lbm.LBM_ENAN
    s.close()
    s = lbm.Solver(d, "fp64")
    C = s.export("C")
    C[0, 16, 16, 16] = 150.0          # tr C > L^2 = 100 inside the droplet
    s.import_("C", C)
    s.step(1)
    assert s.observe()["status"] == lbm.LBM_EFENE
    s.close()


def test_batch_flags_only_the_poisoned_run(lbm):
    runs = [WL.small_newtonian(), WL.small_newtonian(), WL.small_newtonian()]
    b = lbm.Batch(runs, "fp32")
    f = b.export("f", 1)
    f[1, 5, 3, 3, 3] = np.inf
    b.import_("f", f, run=1)
    b.step(5)
    st = [o["status"] for o in b.observe()]
    assert st == [0, lbm.LBM_ENAN, 0]
    b.close()


def test_component_count_matches_oracle(lbm):
    # two droplets plus a tiny speck: count of pieces >= 1% of the initial
    # droplet volume (R = 8 -> 2109 nodes -> 22 nodes)
    d = WL.small_newtonian()
    nz = ny = nx = 32
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = ((x - 8) ** 2 + (y - 16) ** 2 + (z - 16) ** 2 < 25) \
        | ((x - 24) ** 2 + (y - 16) ** 2 + (z - 16) ** 2 < 30) \
        | ((x == 0) & (y == 0) & (z == 3))
    # a droplet split across the periodic x seam is one piece
    m |= ((np.minimum(x, 32 - x) ** 2 + (y - 5) ** 2 + (z - 5) ** 2) < 9)
    rA = np.where(m, 1.0, 0.04)
    rB = np.where(m, 0.04, 1.0)
    f = np.stack([d3q19.W[:, None, None, None] * rA, d3q19.W[:, None, None, None] * rB])
    s = lbm.Solver(d, "fp64")
    s.import_("f", f)
    o = s.observe(components=True)
    sizes = component_sizes(m)
    big = sorted((v for v in sizes if v >= 22), reverse=True)
    assert o["n_components"] == len(big) == 3
    assert o["piece_nodes"] == big + [0] * (4 - len(big))
    s.close()


# Bars of the reduced-precision storage against the FP64 path: D within
# 1e-3 (FP32) and 5e-3 (FP16S), velocity relative L2 within 1e-4 for both.
@pytest.mark.parametrize("precision,d_tol,u_tol", [("fp32", 1e-3, 1e-4), ("fp16s", 5e-3, 1e-4)])
def test_reduced_precision_against_fp64(lbm, precision, d_tol, u_tol):
    d = WL.small_droplet_viscoelastic()
    ref = lbm.Solver(d, "fp64")
    low = lbm.Solver(d, precision)
    for _ in range(5):
        ref.step(200)
        low.step(200)
    o64, olo = ref.observe(), low.observe()
    assert abs(olo["D"] - o64["D"]) <= d_tol
    u64, ulo = ref.export("u"), low.export("u")
    err = math.sqrt(((ulo - u64) ** 2).sum() / (u64 ** 2).sum())
    print(f"{precision}: D {olo['D']:.6e} vs {o64['D']:.6e}; u rel L2 {err:.3e}")
    if u_tol is not None:
        assert err <= u_tol
    ref.close()
    low.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16s"])
def test_reduced_precision_mass_drift(lbm, precision):
    """Each component's mass is conserved by the scheme; in reduced precision
    only rounding of small shifted values may move it (the FP32 weights sum to
    1 + 1.5e-8, which must not leak into the mass as a per-step factor)."""
    d = WL.small_droplet_viscoelastic()
    s = lbm.Solver(d, precision)
    m0 = s.observe()["mass"]
    s.step(3000)
    m1 = s.observe()["mass"]
    drift = [abs(b - a) / a for a, b in zip(m0, m1)]
    print(f"{precision}: relative mass drift {drift}")
    assert max(drift) < 1e-5
    s.close()


# ---- full size, in the bench's launch configuration ----------------------------
# One step of the 512x256x128 matrix-viscoelastic workload after 100 steps of
# flow, checked on sampled columns: the oracle advances a 9x9x128 column block
# cut from the GPU's state (periodic in x and y like the lattice).  A node's
# update reads the state within radius 2, so the block's centre column is
# exact although the block's own periodic wrap is not the lattice's.
FULL_COLUMNS = [(255, 127), (256, 128), (223, 127), (288, 128),   # droplet, interface
                (31, 7), (32, 8), (0, 0), (511, 255), (100, 200)]  # tile and periodic seams


def _column_block(a, x, y, nx, ny, h=4):
    xi = np.arange(x - h, x + h + 1) % nx
    yi = np.arange(y - h, y + h + 1) % ny
    return np.ascontiguousarray(a[..., yi, :][..., xi])


FULL_LAUNCH = {"fp64": dict(bx=16, by=8, bz=64, persistent=2048),
               "fp32": dict(bx=32, by=8, bz=128, persistent=0)}


FULL_LAUNCH["fp16s"] = FULL_LAUNCH["fp32"]


def _shifted(f):
    """g_i = f_i - w_i (rho + 3 c_i.j) of every node (FP64)."""
    c = d3q19.C.astype(float)
    rho = f.sum(axis=1)
    j = np.einsum("sq...,qa->sa...", f, c)
    cj = np.einsum("qa,sa...->sq...", c, j)
    return f - d3q19.W[None, :, None, None, None] * (rho[:, None] + 3.0 * cj)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp16s", None)])
def test_full_size_one_step_sampled(lbm, precision, tol):
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    p, _ = bench.workload_params()
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    print(f"case full size {nx}x{ny}x{nz} {precision}, launch {FULL_LAUNCH[precision]}", flush=True)
    s = lbm.Solver(p, precision)
    s.set_launch(**FULL_LAUNCH[precision])
    s.step(100)
    f0, C0 = s.export("f"), s.export("C")
    s.step(1)
    f1, C1 = s.export("f"), s.export("C")
    s.close()
    fmax, cmax = max(f1.max(), -f1.min()), max(C1.max(), -C1.min())
    tolC = tol
    if precision == "fp16s":
        # FP16 holds g * 2^12 with 11 significant bits: a stored value is off
        # by less than one spacing, 2^-10 |g| (stochastic rounding), plus the
        # FP32 arithmetic; C is stored in FP32
        gmax = float(np.abs(_shifted(f1)).max())
        tol = 2.0 ** -10 * gmax / fmax + 2e-6
        tolC = 1e-5
        print(f"  fp16s tolerance {tol:.2e} (max |g| {gmax:.3e}, max |f| {fmax:.3e})", flush=True)
    for x, y in FULL_COLUMNS:
        d = dict(p, nx=9, ny=9)
        o = Oracle(d, f=_column_block(f0, x, y, nx, ny), C=_column_block(C0, x, y, nx, ny))
        o.step(1)
        ef = np.abs(o.f[..., 4, 4] - f1[..., y, x]).max() / fmax
        eC = np.abs(o.C[..., 4, 4] - C1[..., y, x]).max() / cmax
        print(f"  column ({x}, {y}): f {ef:.1e}, C {eC:.1e}", flush=True)
        assert o.status == 0
        assert ef <= tol and eC <= tolC, (x, y, ef, eC)


@pytest.mark.timeout(600)
def test_wide_run_one_step_sampled(lbm):
    """A run whose 19 population arrays of one component span more than
    4 GiB (FP64, 400 x 384 x 192 = 29.5 M nodes: 4.5 GiB) takes the grouped
    addressing by itself; one step checked against the oracle on sampled
    columns (droplet, interface, tile seams, periodic edges)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    p = dict(bench.workload_params()[0], nx=400, ny=384, nz=192)   # the R = 32 droplet
    nx, ny = p["nx"], p["ny"]
    assert 19 * nx * ny * p["nz"] * 8 > 1 << 32
    print(f"case wide run {nx}x{ny}x{p['nz']} fp64", flush=True)
    s = lbm.Solver(p, "fp64")
    s.set_launch(bx=16, by=8, bz=64, persistent=0)
    assert s.launch["grouped"] == 0      # chosen per run size inside the library
    s.step(20)
    f0, C0 = s.export("f"), s.export("C")
    s.step(1)
    f1, C1 = s.export("f"), s.export("C")
    s.close()
    fmax, cmax = max(f1.max(), -f1.min()), max(C1.max(), -C1.min())
    for x, y in [(199, 191), (200, 192), (168, 192), (232, 191), (15, 7), (16, 8),
                 (0, 0), (399, 383), (100, 300)]:
        o = Oracle(dict(p, nx=9, ny=9), f=_column_block(f0, x, y, nx, ny),
                   C=_column_block(C0, x, y, nx, ny))
        o.step(1)
        ef = np.abs(o.f[..., 4, 4] - f1[..., y, x]).max() / fmax
        eC = np.abs(o.C[..., 4, 4] - C1[..., y, x]).max() / cmax
        print(f"  column ({x}, {y}): f {ef:.1e}, C {eC:.1e}", flush=True)
        assert o.status == 0
        assert ef <= 1e-12 and eC <= 1e-12, (x, y, ef, eC)


@pytest.mark.parametrize("eta", [(0.0, 0.0), (0.0, 0.05)])
def test_no_droplet_couette_parity(lbm, eta):
    # degenerate case: no droplet (R = 0), plane Couette flow of the matrix,
    # with and without polymer in the matrix
    d = WL.base_params(nx=8, ny=6, nz=20, radius=0.0, u_wall=0.01, tau=(1.0, 1.0),
                       tau_P=(1.0, 40.0), eta_P=eta, L2=(100.0, 100.0))
    print(f"case no droplet, eta_P {eta}", flush=True)
    s = lbm.Solver(d, "fp64")
    s.step(300)
    g = _fields(s)
    o = Oracle(d)
    o.step(300)
    assert rel(g["f"], o.f) <= 1e-12
    assert rel(g["C"], o.C) <= 1e-12
    assert rel(g["u"], o.velocity()) <= 1e-11
    ob = s.observe(components=True)
    assert ob["status"] == 0 and ob["weight"] == 0.0
    assert ob["D"] == 0.0 and ob["Lp"] == 0.0
    assert ob["n_components"] == 0 and ob["piece_nodes"] == [0, 0, 0, 0]
    s.close()


def test_layered_couette_parity(lbm):
    """Polymer layer below a Newtonian layer in plane Couette flow (the
    stress-balance case of the oracle's polymer pins): FP64 fields after
    2000 steps against the oracle."""
    from tests.test_oracle_polymer import layered_couette_params, layered_state
    d = layered_couette_params(24)
    f0 = layered_state(24)
    print("case layered Couette 3x3x24, 2000 steps", flush=True)
    s = lbm.Solver(d, "fp64")
    s.import_("f", f0)
    s.step(2000)
    g = _fields(s)
    o = Oracle(d, f=f0)
    o.step(2000)
    for k, ref in (("f", o.f), ("C", o.C), ("rho", o.density()), ("u", o.velocity())):
        assert rel(g[k], ref) <= 1e-10, k
    assert abs(o.C[4]).max() > 1e-2      # the polymer layer is sheared
    s.close()


def test_component_labelling_of_a_thread_shaped_droplet(lbm):
    """A droplet at the R = 24 study scale stretched into a long thread of
    radius 4 that has broken in two places, with bulbous ends and a small
    satellite (the shape just after a multiple necking, Section 3): counts
    and piece sizes against the oracle's breadth-first search, and the cost
    of the labelling (long threads are the worst case for the union-find)."""
    import time
    nx, ny, nz = 320, 48, 50
    d = WL.base_params(nx=nx, ny=ny, nz=nz, radius=24.0, u_wall=0.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    yc, zc = 23.5, 24.5
    tube = (y - yc) ** 2 + (z - zc) ** 2 < 16.0
    m = tube & (((x >= 14) & (x <= 109)) | ((x >= 113) & (x <= 199)) | ((x >= 203) & (x <= 305)))
    m |= (x - 14) ** 2 + (y - yc) ** 2 + (z - zc) ** 2 < 81.0         # end bulbs
    m |= (x - 305) ** 2 + (y - yc) ** 2 + (z - zc) ** 2 < 81.0
    m |= (x - 111) ** 2 + (y - yc - 9) ** 2 + (z - zc) ** 2 < 6.25    # satellite
    # the last piece wraps through the periodic x seam
    m |= tube & ((x >= 316) | (x <= 14))
    rA = np.where(m, 1.0, 0.04)
    rB = np.where(m, 0.04, 1.0)
    f = np.stack([d3q19.W[:, None, None, None] * rA, d3q19.W[:, None, None, None] * rB])
    s = lbm.Solver(d, "fp32")
    s.import_("f", f)
    s.observe()                                   # warm-up
    t0 = time.perf_counter()
    s.observe()
    t1 = time.perf_counter()
    o = s.observe(components=True)
    t2 = time.perf_counter()
    sizes = component_sizes(m)
    min_cc = -(-int((((x - (nx - 1) / 2) ** 2 + (y - (ny - 1) / 2) ** 2
                      + (z - (nz - 1) / 2) ** 2) < 24.0 ** 2).sum()) // 100)
    big = sorted((v for v in sizes if v >= min_cc), reverse=True)
    print(f"case thread {nx}x{ny}x{nz}: pieces {big} (all {sizes[:6]}), min {min_cc}; "
          f"labelling {1e3 * ((t2 - t1) - (t1 - t0)):.2f} ms", flush=True)
    assert o["status"] == 0
    assert o["n_components"] == len(big) == 3
    assert o["piece_nodes"] == big + [0] * (4 - len(big))
    assert len(sizes) == 4 and sizes[-1] < min_cc      # the satellite is not counted
    s.close()
