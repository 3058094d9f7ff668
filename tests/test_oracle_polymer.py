"""Pins of the oracle's polymer feedback (Section 2, Eqs. (1) and (3): the
body force (eta_P/tau_P) div[f C] acting in the polymer phase) against
results fixed outside the oracle's own formulas:

  * manufactured conformation fields whose centred divergence is known in
    closed form (trigonometric profiles, exact for the centred difference),
    including a profile that is exactly consistent with the zero-gradient
    ghost planes at the walls;
  * a polymer at rest (C = I) exerts no force, whatever the phase indicator
    does across an interface;
  * the split of the force over the two components adds up to the whole;
  * a layered plane Couette flow, polymer phase below and Newtonian phase
    above: in steady state the shear stress (solvent plus polymer) is the
    same in both layers, so the bulk shear rates stand in the ratio of the
    layers' total viscosities, eta_s/(eta_s + eta_P) in the Oldroyd-B limit
    (Eq. (6) with L^2 -> infinity gives a polymer shear stress eta_P * shear
    rate);
  * the physical velocity is the time-centred momentum: half-way between
    the momentum before and after the collision.
"""
import math

import numpy as np
import pytest

import workloads as WL
from oracle.d3q19 import Q, W
from oracle.solver import (Oracle, Params, collide, forces, moments,
                           velocities)

# component order of C: xx yy zz xy xz yz


def _uniform_rho(shape, rho_major=1.0, rho_minor=0.04, polymer="B"):
    """Densities with the polymer phase's component the majority everywhere,
    so that the phase indicator clamps to 1 and the Shan-Chen force is
    zero (uniform densities)."""
    rp = np.full(shape, rho_major)
    rq = np.full(shape, rho_minor)
    return np.stack([rq, rp]) if polymer == "B" else np.stack([rp, rq])


def _params(shape, eta_P=0.03, tau_P=20.0, L2=1e12, phase="B"):
    nz, ny, nx = shape
    eta = (0.0, eta_P) if phase == "B" else (eta_P, 0.0)
    return Params(WL.base_params(nx=nx, ny=ny, nz=nz, radius=0.0,
                                 tau_P=(tau_P, tau_P), eta_P=eta, L2=(L2, L2)))


def _identity_C(shape):
    C = np.zeros((6,) + shape)
    C[0] = C[1] = C[2] = 1.0
    return C


def test_polymer_force_of_a_sinusoidal_shear_conformation():
    """C = I + a sin(2 pi x/nx)(e_x e_z + e_z e_x): tr C = 3, so the
    Peterlin factor is exactly 1 and T_xz = (eta_P/tau_P) a sin(2 pi x/nx).
    The centred divergence is then F_z = (eta_P/tau_P) a sin(2 pi/nx)
    cos(2 pi x/nx), and F_x = F_y = 0 (T varies along x only and T_xx = 0).
    A sign error, a missing 1/2, or a transposed index of the stress
    (F_x from dT_xz/dx) fails this."""
    nz, ny, nx = 4, 3, 16
    shape = (nz, ny, nx)
    eta_P, tau_P, a = 0.03, 20.0, 0.37
    prm = _params(shape, eta_P, tau_P, L2=100.0)
    rho = _uniform_rho(shape)
    C = _identity_C(shape)
    x = np.arange(nx)[None, None, :] * np.ones(shape)
    C[4] = a * np.sin(2 * math.pi * x / nx)
    FA, FB = forces(rho, C, prm)
    F = FA + FB
    e = eta_P / tau_P
    want_z = e * a * math.sin(2 * math.pi / nx) * np.cos(2 * math.pi * x / nx)
    assert np.abs(F[2] - want_z).max() <= 1e-16
    assert np.abs(F[0]).max() <= 1e-18 and np.abs(F[1]).max() <= 1e-18
    assert np.abs(want_z).max() > 1e-4     # not a trivial zero


def test_polymer_force_of_a_normal_stress_profile_in_y():
    """C_yy = 1 + b cos(2 pi y/ny) in the Oldroyd-B limit (f -> 1):
    T_yy = (eta_P/tau_P) b cos(2 pi y/ny) and the centred divergence is
    F_y = -(eta_P/tau_P) b sin(2 pi/ny) sin(2 pi y/ny); F_x = F_z = 0."""
    nz, ny, nx = 3, 12, 4
    shape = (nz, ny, nx)
    eta_P, tau_P, b = 0.05, 8.0, 0.6
    prm = _params(shape, eta_P, tau_P, L2=1e14)
    rho = _uniform_rho(shape)
    C = _identity_C(shape)
    y = np.arange(ny)[None, :, None] * np.ones(shape)
    C[1] = 1.0 + b * np.cos(2 * math.pi * y / ny)
    FA, FB = forces(rho, C, prm)
    F = FA + FB
    e = eta_P / tau_P
    want_y = -e * b * math.sin(2 * math.pi / ny) * np.sin(2 * math.pi * y / ny)
    # f - 1 is of order tr(C)/L^2 ~ 1e-14 here
    assert np.abs(F[1] - want_y).max() <= 1e-14 * np.abs(want_y).max() + 1e-17
    assert np.abs(F[0]).max() <= 1e-18 and np.abs(F[2]).max() <= 1e-18


def test_polymer_force_at_the_walls_uses_zero_gradient_ghosts():
    """C_xz(z) = a cos(pi (z + 1/2)/nz) is even about both wall planes
    (z = -1/2 and z = nz - 1/2), so it is exactly the profile that the
    zero-gradient ghost rule continues; its centred divergence at every
    plane, the two next to the walls included, is
    F_x = -(eta_P/tau_P) a sin(pi/nz) sin(pi (z + 1/2)/nz)."""
    nz, ny, nx = 10, 3, 4
    shape = (nz, ny, nx)
    eta_P, tau_P, a = 0.04, 15.0, 0.5
    prm = _params(shape, eta_P, tau_P, L2=100.0)
    rho = _uniform_rho(shape)
    C = _identity_C(shape)
    z = np.arange(nz)[:, None, None] * np.ones(shape)
    C[4] = a * np.cos(math.pi * (z + 0.5) / nz)
    FA, FB = forces(rho, C, prm)
    F = FA + FB
    e = eta_P / tau_P
    want_x = -e * a * math.sin(math.pi / nz) * np.sin(math.pi * (z + 0.5) / nz)
    assert np.abs(F[0] - want_x).max() <= 1e-16
    assert np.abs(F[1]).max() <= 1e-18 and np.abs(F[2]).max() <= 1e-18


@pytest.mark.parametrize("L2", [10.0, 100.0])
def test_isotropic_conformation_stress_through_the_peterlin_factor(L2):
    """C = c(x) I: f = (L^2 - 3)/(L^2 - 3c), so
    f c - 1 = L^2 (c - 1)/(L^2 - 3c) (simplified by hand), and the force is
    F_x = (eta_P/tau_P)[g(x+1) - g(x-1)]/2 with g = L^2 (c-1)/(L^2-3c)."""
    nz, ny, nx = 3, 3, 10
    shape = (nz, ny, nx)
    eta_P, tau_P = 0.02, 5.0
    prm = _params(shape, eta_P, tau_P, L2=L2)
    rho = _uniform_rho(shape)
    rng = np.random.default_rng(3)
    c1 = rng.uniform(0.6, 2.0, size=nx)
    C = np.zeros((6,) + shape)
    for k in range(3):
        C[k] = c1[None, None, :]
    FA, FB = forces(rho, C, prm)
    F = FA + FB
    g = L2 * (c1 - 1.0) / (L2 - 3.0 * c1)
    want = (eta_P / tau_P) * 0.5 * (np.roll(g, -1) - np.roll(g, 1))
    assert np.allclose(F[0], want[None, None, :], rtol=1e-13, atol=1e-18)
    assert np.abs(F[1]).max() <= 1e-18 and np.abs(F[2]).max() <= 1e-18


def test_polymer_at_rest_exerts_no_force_across_an_interface():
    """C = I (no deformation): the polymer stress vanishes wherever the
    polymer is, and with it the force, even where the phase indicator
    varies across an interface.  (A stress of f C without the -I would
    leave a force (eta_P/tau_P) grad chi at the interface.)"""
    nz, ny, nx = 12, 3, 4
    shape = (nz, ny, nx)
    prm = _params(shape, 0.05, 10.0, L2=50.0, phase="A")
    z = np.arange(nz)[:, None, None] * np.ones(shape)
    xa = 0.5 * (1.0 + np.tanh((z - 5.5) / 1.5))    # A fraction across z
    rho = np.stack([1.04 * xa, 1.04 * (1.0 - xa)])
    C = _identity_C(shape)
    FA0, FB0 = forces(rho, C, prm)
    prm_n = _params(shape, 0.0, 10.0, L2=50.0, phase="A")
    FAn, FBn = forces(rho, C, prm_n)               # Shan-Chen force alone
    assert np.abs(FA0 - FAn).max() == 0.0 and np.abs(FB0 - FBn).max() == 0.0


def test_polymer_force_split_adds_up_and_follows_mass_fraction():
    """With uniform densities the Shan-Chen force vanishes, so the two
    component forces are the polymer force split by mass fraction; they
    add up to the whole force (momentum of the polymer body force).  At a
    mass fraction between the indicator's bounds the force is scaled by the
    rescaled fraction chi = (x_p - chi_lo)/(chi_hi - chi_lo)."""
    nz, ny, nx = 4, 3, 16
    shape = (nz, ny, nx)
    eta_P, tau_P, a = 0.03, 20.0, 0.2
    prm = _params(shape, eta_P, tau_P, L2=100.0)
    C = _identity_C(shape)
    x = np.arange(nx)[None, None, :] * np.ones(shape)
    C[4] = a * np.sin(2 * math.pi * x / nx)
    e = eta_P / tau_P
    Fz = e * a * math.sin(2 * math.pi / nx) * np.cos(2 * math.pi * x / nx)
    # polymer component (B) above the upper bound: chi = 1
    FA, FB = forces(_uniform_rho(shape, 0.95, 0.05), C, prm)
    assert np.abs(FA[2] + FB[2] - Fz).max() <= 1e-16
    assert np.allclose(FA[2], 0.05 * Fz, rtol=1e-14, atol=1e-18)
    assert np.allclose(FB[2], 0.95 * Fz, rtol=1e-14, atol=1e-18)
    # B fraction 0.6: chi = (0.6 - lo)/(hi - lo), lo/hi the mean-field
    # coexistence fractions at G = 0.9, rho_tot = 1.04 (0.0917 / 0.9083)
    FA, FB = forces(_uniform_rho(shape, 0.6, 0.4), C, prm)
    chi = (0.6 - prm.chi_lo) / (prm.chi_hi - prm.chi_lo)
    assert 0.6 < chi < 0.65
    assert np.allclose(FA[2] + FB[2], chi * Fz, rtol=1e-13, atol=1e-18)
    assert np.allclose(FB[2], 0.6 * chi * Fz, rtol=1e-13, atol=1e-18)
    # polymer component below the lower bound: no force
    FA, FB = forces(_uniform_rho(shape, 0.05, 0.95), C, prm)
    assert np.abs(FA).max() == 0.0 and np.abs(FB).max() == 0.0


def test_physical_velocity_is_the_time_centred_momentum():
    """u rho = (j + j*)/2 node by node, with j* the momentum after the
    collision (the collision adds the force F_A + F_B to the momentum):
    the physical velocity sits half-way through the step's forcing."""
    shape = (6, 5, 7)
    nz, ny, nx = shape
    p = WL.base_params(nx=nx, ny=ny, nz=nz, u_wall=0.01, tau=(0.8, 1.3),
                       tau_P=(20.0, 1.0), eta_P=(0.05, 0.0))
    prm = Params(p)
    f = WL.random_populations(shape, W, seed=21)
    C = WL.random_conformation(shape, seed=22)
    rho, j = moments(f)
    FA, FB = forces(rho, C, prm)
    ueqA, ueqB, u = velocities(rho, j, FA, FB, prm)
    fs = collide(f, rho, ueqA, ueqB, prm)
    _, js = moments(fs)
    mid = 0.5 * ((j[0] + j[1]) + (js[0] + js[1]))
    assert np.abs(u * (rho[0] + rho[1]) - mid).max() <= 1e-15 * np.abs(mid).max()
    assert np.abs(FA + FB).max() > 1e-4


# --------------------------------------------------------------------------
# layered plane Couette flow with polymer in the lower layer
# --------------------------------------------------------------------------
def layered_couette_params(nz=24):
    """Both components relax with tau = 1 (the solvent viscosity is then
    rho c_s^2 (tau - 1/2) in either layer), polymer in component A with
    eta_P = 1.04/6 (the solvent viscosity at the reference density 1.04),
    tau_P = 50 and L^2 = 1e8 (Oldroyd-B limit), walls at -+0.01."""
    eta_P = 1.04 * 0.5 / 3.0
    return WL.base_params(nx=3, ny=3, nz=nz, radius=0.0, u_wall=0.01,
                          tau=(1.0, 1.0), tau_P=(50.0, 1.0),
                          eta_P=(eta_P, 0.0), L2=(1e8, 1e8))


def layered_state(nz=24):
    """Component A (the polymer phase) fills the lower half of the gap,
    component B the upper half; flat interface, fluid at rest."""
    lower = (np.arange(nz) < nz // 2)[:, None, None] * np.ones((nz, 3, 3), bool)
    rA = np.where(lower, 0.9446, 0.0954)
    rB = np.where(lower, 0.0954, 0.9446)
    return np.stack([W[:, None, None, None] * rA, W[:, None, None, None] * rB])


def test_layered_couette_stress_balance():
    nz = 24
    p = layered_couette_params(nz)
    o = Oracle(p, f=layered_state(nz))
    o.step(5000)
    assert o.status == 0
    u = o.velocity()[0, :, 1, 1]
    rho = o.density()[:, :, 1, 1]
    Cxz = o.C[4, :, 1, 1]
    lower = slice(1, 6)        # bulk of the polymer layer (interface at ~11.5)
    upper = slice(16, 22)      # bulk of the Newtonian layer
    g = np.diff(u)             # shear rate between planes z and z + 1
    gl, gu = g[lower], g[upper]
    # linear in each bulk layer
    assert np.ptp(gl) <= 1e-3 * gl.mean() and np.ptp(gu) <= 1e-3 * gu.mean()
    eta_s_l = (rho[0, 3] + rho[1, 3]) * 0.5 / 3.0
    eta_s_u = (rho[0, 19] + rho[1, 19]) * 0.5 / 3.0
    eta_P = p["eta_P"][0]
    # slopes in the ratio of the total viscosities of the layers
    ratio = gl.mean() / gu.mean()
    want = eta_s_u / (eta_s_l + eta_P)
    assert abs(ratio / want - 1.0) <= 1e-2, (ratio, want)
    # Oldroyd-B steady shear: C_xz = tau_P * shear rate in the polymer layer
    assert abs(Cxz[3] / (50.0 * gl.mean()) - 1.0) <= 1e-2
    # the shear stress is the same in both layers
    s_l = eta_s_l * gl.mean() + (eta_P / 50.0) * Cxz[3]
    s_u = eta_s_u * gu.mean()
    assert abs(s_l / s_u - 1.0) <= 1e-2, (s_l, s_u)
    # the feedback is a real effect: without polymer the slopes would match
    assert ratio < 0.6
