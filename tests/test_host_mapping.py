"""Host logic of the physical -> lattice mapping (physics.py), the sweep's
reachable-Ca window and box (sweep.py) and the autotuner's candidates: the
returned lattice parameters reproduce the dimensionless groups they were
asked for (Ca = eta_M gamma_dot R / sigma, gamma_dot = 2 U_w / W, the
viscosity ratio on total viscosity, the polymer fraction, De = tau_P
gamma_dot), whichever phase carries the polymer."""
import os
import re

import pytest

from paper_1411_2181_amd import autotune, physics, sweep


def _etas(p):
    eta_A, eta_B = (physics.eta_of_tau(t) for t in p["tau"])
    return eta_A, eta_B, p["eta_P"]


@pytest.mark.parametrize("phase,lam,fraction,De", [("N", 1.0, 0.0, 0.0), ("N", 0.5, 0.0, 0.0),
                                                   ("DV", 4 / 3, 0.4, 1.0), ("DV", 1.0, 0.2, 0.5),
                                                   ("MV", 0.5, 0.4, 1.0)])
def test_lattice_params_reproduce_the_groups(phase, lam, fraction, De):
    nx, ny, nz, R, Ca = 144, 72, 96, 24.0, 0.15
    p, info = physics.lattice_params(nx, ny, nz, R=R, Ca=Ca, De=De, lam=lam, phase=phase,
                                     L2=100.0, fraction=fraction, tau_matrix=1.5, u_max=0.19)
    eta_A, eta_B, eta_P = _etas(p)
    gdot = 2.0 * p["u_wall"] / nz
    assert gdot == pytest.approx(info["gamma_dot"], rel=1e-12)
    if phase == "MV":
        eta_M = eta_B + eta_P[1]
        assert eta_P[1] / eta_M == pytest.approx(fraction, rel=1e-12)
        assert eta_A / eta_M == pytest.approx(lam, rel=1e-12)
    else:
        eta_M = eta_B
        eta_d = eta_A + eta_P[0]
        assert eta_d / eta_M == pytest.approx(lam, rel=1e-12)
        if phase == "DV":
            assert eta_P[0] / eta_d == pytest.approx(fraction, rel=1e-12)
    assert info["eta_M"] == pytest.approx(eta_M, rel=1e-12)
    assert eta_M * gdot * R / info["sigma"] == pytest.approx(Ca, rel=1e-12)
    assert info["tau_em"] == pytest.approx(R * eta_M / info["sigma"], rel=1e-12)
    if De > 0:
        assert p["tau_P"][0] * gdot == pytest.approx(De, rel=1e-12)
    assert p["u_wall"] <= 0.19 and max(p["tau"]) <= physics.TAU_MAX


def test_viscosity_tau_inverse_and_taylor_law():
    for tau in (0.6, 1.0, 1.24, 1.5):
        assert physics.tau_of_eta(physics.eta_of_tau(tau)) == pytest.approx(tau, rel=1e-14)
    assert physics.eta_of_tau(1.5) == pytest.approx(1.04 / 3.0, rel=1e-14)
    assert physics.taylor_deformation(0.1, 1.0) == pytest.approx(0.1 * 35.0 / 32.0, rel=1e-14)
    assert physics.taylor_deformation(0.1, 0.0) == pytest.approx(0.1, rel=1e-14)


def test_reachable_ca_is_the_wall_speed_cap():
    for c, lam, De, f in ((0.5, 4 / 3, 1.0, 0.4), (0.6, 1.0, 0.5, 0.2), (0.45, 0.8, 0.0, 0.0)):
        hi = sweep.ca_max(24.0, c, lam, De, f)
        p, _ = sweep.lattice(sweep.RunSpec(24.0, c, hi, De, lam, 100.0, f))
        assert p["u_wall"] == pytest.approx(sweep.U_MAX, rel=1e-9)
        nx, ny, nz = sweep.box(24.0, c)
        assert (nx, ny) == (round(sweep.BOX_X * 24), 72) and nz == round(48 / c)


def test_autotune_candidates_are_compiled_shapes():
    with open(os.path.join(os.path.dirname(autotune.__file__), "csrc", "lbm_step.hip")) as fh:
        src = fh.read()
    compiled = {tuple(map(int, m)) for m in re.findall(r"M\((\d+), (\d+)\)",
                                                       src[src.index("#define LBM_FOR_SHAPES"):][:200])}
    cands = autotune.candidates(128)
    assert cands and all((c["bx"], c["by"]) in compiled for c in cands)
    assert all(c["bx"] * c["by"] <= 1024 and c["bz"] >= 1 for c in cands)
    # small lattices keep at least the smallest z block
    assert all(c["bz"] <= 8 for c in autotune.candidates(4))
