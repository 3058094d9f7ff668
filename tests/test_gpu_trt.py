"""The two-relaxation-time collision (tau_minus in lbm_params) through the C
ABI against the oracle's, whose collision is pinned by tests/test_oracle_trt.py.
FP64 random states with ragged tiles and wall links: <= 1e-12 after 10 steps;
the 32^3 viscoelastic droplet cases: <= 1e-10 after 1000 steps; FP32 and
FP16S at their storage bars; a batch that mixes BGK and TRT runs reproduces
each run's own launch bit for bit; Couette flow stays exactly linear."""
import numpy as np
import pytest

import workloads as WL
from oracle import d3q19
from oracle.observables import observe
from oracle.solver import Oracle
from tests import oracle_pool

pytestmark = pytest.mark.gpu

TM = (0.7, 1.9)   # tau^- of A and B: Lambda far from the BGK values


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


def _trt(d, tm=TM):
    return dict(d, tau_minus=tm)


TRT_CASES = {"droplet_visc": lambda: _trt(WL.small_droplet_viscoelastic(), (0.9, 0.75)),
             "matrix_visc": lambda: _trt(WL.small_matrix_viscoelastic(), (1.3, 0.8))}


@pytest.fixture(scope="module")
def oracle_1000():
    return {k: oracle_pool.submit(fn(), 1000) for k, fn in TRT_CASES.items()}


@pytest.mark.parametrize("shape_xyz", [(17, 9, 12), (33, 5, 40)])
@pytest.mark.parametrize("visc", ["none", "A", "B"])
def test_trt_random_state_ragged_parity(lbm, shape_xyz, visc):
    nx, ny, nz = shape_xyz
    eta = {"none": (0.0, 0.0), "A": (0.05, 0.0), "B": (0.0, 0.05)}[visc]
    d = _trt(WL.base_params(nx=nx, ny=ny, nz=nz, radius=3.0, u_wall=0.02, tau=(0.8, 1.3),
                            tau_P=(20.0, 30.0), eta_P=eta, L2=(60.0, 80.0)))
    print(f"case TRT ragged {shape_xyz} visc={visc}", flush=True)
    f0 = WL.random_populations((nz, ny, nx), d3q19.W, seed=17)
    C0 = WL.random_conformation((nz, ny, nx), seed=18)
    s = lbm.Solver(d, "fp64")
    s.import_("f", f0)
    s.import_("C", C0)
    s.step(10)
    o = Oracle(d, f=f0, C=C0)
    o.step(10)
    assert rel(s.export("f"), o.f) <= 1e-12
    assert rel(s.export("C"), o.C) <= 1e-12
    assert rel(s.export("u"), o.velocity()) <= 1e-11
    # the two collisions differ here (the check is not trivial)
    b = Oracle(dict(d, tau_minus=(0.0, 0.0)), f=f0, C=C0)
    b.step(10)
    assert rel(b.f, o.f) > 1e-4
    s.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", list(TRT_CASES))
def test_trt_droplet_1000_steps_parity(lbm, oracle_1000, case):
    d = TRT_CASES[case]()
    print(f"case TRT 32^3 {case} 1000 steps", flush=True)
    s = lbm.Solver(d, "fp64")
    s.step(1000)
    o = oracle_1000[case].result()
    for k in ("f", "C", "rho", "u"):
        assert rel(s.export(k), o[k]) <= 1e-10, k
    go = s.observe()
    assert abs(go["D"] - o["obs"]["D"]) <= 1e-10 * max(abs(o["obs"]["D"]), 1e-6)
    assert go["status"] == 0 and o["status"] == 0 and go["D"] > 1e-3
    s.close()


def test_trt_reduced_precision(lbm):
    """FP32 against the oracle (1e-5 on f after 200 steps) and FP16S against
    the FP64 path (velocity rel. L2 <= 1e-4, the storage bar) with a common
    tau^- = 1.  (An odd-moment time below 1 thins the minority density
    inside the droplet, as BGK's tau < 1 does, and the FP16 shifted values
    of that component lose precision: 8e-4 at tau^- = (0.9, 0.75).)"""
    d = TRT_CASES["droplet_visc"]()
    print("case TRT fp32 / fp16s 32^3", flush=True)
    o = Oracle(d)
    o.step(200)
    s = lbm.Solver(d, "fp32")
    s.step(200)
    assert rel(s.export("f"), o.f) <= 1e-5
    s.close()
    d = dict(d, tau_minus=(1.0, 1.0))
    ref = lbm.Solver(d, "fp64")
    h = lbm.Solver(d, "fp16s")
    ref.step(1000)
    h.step(1000)
    ur, uh = ref.export("u"), h.export("u")
    assert np.sqrt(((uh - ur) ** 2).sum() / (ur ** 2).sum()) <= 1e-4
    ref.close()
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_batch_of_bgk_and_trt_runs_equals_single_runs(lbm, precision):
    """The batch takes the TRT instance for all of its runs; a BGK run in it
    (tau^- = tau) must still match its own BGK launch bit for bit."""
    runs = [WL.base_params(nx=20, ny=24, nz=18, radius=5.0, tau=(1.0, 0.8),
                           tau_P=(1.0, 50.0), eta_P=(0.0, 0.05), u_wall=0.01),
            _trt(WL.base_params(nx=17, ny=9, nz=12, radius=3.0, u_wall=0.02)),
            _trt(WL.small_droplet_viscoelastic(), (0.9, 0.75))]
    steps = [23, 31, 17]
    print(f"case TRT/BGK batch {precision}", flush=True)
    b = lbm.Batch(runs, precision)
    b.step(steps)
    for r, d in enumerate(runs):
        s = lbm.Solver(d, precision)
        s.step(steps[r])
        assert np.array_equal(b.export("f", r), s.export("f")), r
        assert np.array_equal(b.export("C", r), s.export("C")), r
        s.close()
    b.close()


def test_trt_launch_shapes_bit_identical(lbm):
    d = _trt(WL.base_params(nx=40, ny=20, nz=14, radius=4.0, u_wall=0.02, tau=(0.9, 1.2),
                            tau_P=(1.0, 30.0), eta_P=(0.0, 0.05)))
    ref = None
    for shape in [dict(bx=16, by=8, bz=1), dict(bx=32, by=8, bz=0), dict(bx=8, by=16, bz=5, persistent=8)]:
        s = lbm.Solver(d, "fp32")
        s.set_launch(**shape)
        s.step(12)
        out = (s.export("f"), s.export("C"))
        s.close()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), shape


def test_trt_couette_is_linear(lbm):
    """Plane Couette flow with unequal rates: the linear profile through the
    half-way walls is exact for any Lambda (FP64, no droplet)."""
    nz, uw = 16, 0.01
    d = _trt(WL.base_params(nx=16, ny=8, nz=nz, radius=0.0, u_wall=uw, rho_major=1.0,
                            rho_minor=1.0, G=0.0, tau=(1.6, 1.6)), (0.6, 0.6))
    s = lbm.Solver(d, "fp64")
    s.step(6000)
    u = s.export("u")
    z = np.arange(nz)
    want = uw * (2 * z + 1 - nz) / nz
    assert np.abs(u[0] - want[:, None, None]).max() <= 1e-11 * uw
    assert np.abs(u[1]).max() <= 1e-12 * uw and np.abs(u[2]).max() <= 1e-12 * uw
    s.close()
