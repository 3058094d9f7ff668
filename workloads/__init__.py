"""Seeded synthetic workloads shared by the tests, the bench and the smoke check.

This module holds inputs only: lattice sizes and parameter sets of the
confined-shear droplet problem (a sphere of radius R at mid-gap between two
walls moving at +/-U_w along x, periodic in x and y), the seeded draws of the
batched Ca-sweep sampler, and seeded random arrays used as initial states in
parity tests.  It contains none of the method's arithmetic: no lattice
weights, no equilibria, no forces.  Both the CPU oracle and the HIP library
receive the values produced here unchanged.

Parameter dictionaries use the field names of ``lbm_params`` in
``include/lbmve.h``:

    nx, ny, nz            fluid nodes; the walls lie half a link outside z=0
                          and z=nz-1, so the gap is W = nz
    u_wall                top wall moves at +u_wall, bottom wall at -u_wall (x)
    radius, cx, cy, cz    droplet; cx < 0 selects the box centre
    rho_major, rho_minor  component densities outside/inside the sphere
    G                     Shan-Chen coupling between the two components
    tau                   (tau_A, tau_B) BGK relaxation times; A is the droplet
                          component, B the matrix component
    tau_minus             (tau^-_A, tau^-_B) antisymmetric relaxation times of
                          the two-relaxation-time collision; 0 = tau (BGK)
    tau_P, eta_P, L2      per-phase FENE-P parameters (A, B); a phase is
                          viscoelastic when its eta_P > 0
    chi_lo, chi_hi        bounds of the polymer-phase indicator (0 = default)
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ----------------------------------------------------------------------------
# Base parameter set: the small Newtonian case of the confined-shear set-up,
# 32^3 lattice, walls at -1/2 and 31.5 (W = 32), U_w = 0.005, G = 0.9,
# densities 1.0 / 0.04 swapped inside a centred sphere of radius 8, tau = 1.
# ----------------------------------------------------------------------------
_BASE = dict(
    nx=32, ny=32, nz=32,
    u_wall=0.005,
    radius=8.0, cx=-1.0, cy=-1.0, cz=-1.0,
    rho_major=1.0, rho_minor=0.04,
    G=0.9,
    tau=(1.0, 1.0),
    tau_P=(1.0, 1.0), eta_P=(0.0, 0.0), L2=(100.0, 100.0),
    chi_lo=0.0, chi_hi=0.0,
    tau_minus=(0.0, 0.0),
)


def base_params(**overrides) -> dict:
    p = copy.deepcopy(_BASE)
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    return p


def small_newtonian() -> dict:
    """32^3, FP64 Newtonian/Newtonian case (2000-step parity run)."""
    return base_params()


def small_droplet_viscoelastic() -> dict:
    """32^3 case with FENE-P in the droplet phase: L^2 = 100, tau_P = 200,
    polymer fraction 0.4 of the droplet viscosity, tau_A = 0.8 so that the
    total droplet viscosity equals the matrix viscosity (lambda = 1).

    eta_s = rho_ref (tau - 1/2)/3 with rho_ref = 1.04: eta_B(tau=1) = 0.17333;
    eta_A(tau=0.8) = 0.104 = 0.6 eta_B; eta_P = 0.4 eta_B = 0.069333.
    """
    rho_ref = 1.04
    eta_B = rho_ref * (1.0 - 0.5) / 3.0
    return base_params(tau=(0.8, 1.0), tau_P=(200.0, 1.0),
                       eta_P=(0.4 * eta_B, 0.0), L2=(100.0, 100.0))


def small_matrix_viscoelastic() -> dict:
    """Mirror of the droplet-viscoelastic case: FENE-P in the matrix phase."""
    rho_ref = 1.04
    eta_A = rho_ref * (1.0 - 0.5) / 3.0
    return base_params(tau=(1.0, 0.8), tau_P=(1.0, 200.0),
                       eta_P=(0.0, 0.4 * eta_A), L2=(100.0, 100.0))


# ----------------------------------------------------------------------------
# Larger single-run workloads (physical description; lattice values such as
# U_w and tau_P follow from Ca, De and the surface tension, mapped by the
# library's host driver).
# ----------------------------------------------------------------------------
def viscoelastic_droplet_192() -> dict:
    """192x96x64 (W=64), R=16 centred, FENE-P in the droplet (L^2=100,
    polymer fraction 0.4), lambda=1 (tau_B=1, tau_A=0.8); De in {0.5,1,2},
    Ca in {0.1,0.2,0.3}; FP32 storage; 20000 steps."""
    return dict(nx=192, ny=96, nz=64, radius=16.0, phase="DV", L2=100.0,
                polymer_fraction=0.4, lam=1.0, De=(0.5, 1.0, 2.0),
                Ca=(0.1, 0.2, 0.3), steps=20000)


def matrix_viscoelastic_512() -> dict:
    """512x256x128 (W=128), R=32 (2R/W=0.5) centred, FENE-P in the matrix
    (L^2=400, De=1, polymer fraction 0.4), lambda in {0.5, 2}, Ca=0.25;
    50000 steps; FP32 and FP16 shift-stored populations."""
    return dict(nx=512, ny=256, nz=128, radius=32.0, phase="MV", L2=400.0,
                polymer_fraction=0.4, lam=(0.5, 2.0), De=1.0, Ca=0.25,
                steps=50000)


def sweep_sampler(k: int, base_seed: int = 1234) -> dict:
    """Physical parameters of run k of the batched Ca sweep.

    R ~ U[8,20]; confinement c in {0.3,0.5,0.7}; box (6R, 3R, 2R/c) rounded;
    Ca ~ U[0.05,0.5]; De in {0,0.5,1,2}; lambda in {0.5,1,2}; droplet phase
    viscoelastic; L^2 = 100; polymer fraction 0.4.
    """
    rng = np.random.default_rng(base_seed + k)
    R = float(rng.uniform(8.0, 20.0))
    c = float(rng.choice([0.3, 0.5, 0.7]))
    Ca = float(rng.uniform(0.05, 0.5))
    De = float(rng.choice([0.0, 0.5, 1.0, 2.0]))
    lam = float(rng.choice([0.5, 1.0, 2.0]))
    nx = int(round(6 * R))
    ny = int(round(3 * R))
    nz = int(round(2 * R / c))
    return dict(k=k, seed=base_seed + k, R=R, confinement=c, Ca=Ca, De=De,
                lam=lam, nx=nx, ny=ny, nz=nz, phase="DV", L2=100.0,
                polymer_fraction=0.4)


def surrogate_sampler(k: int, base_seed: int = 98765) -> dict:
    """Training-run sampler for the surrogate: the sweep sampler with L^2 in
    {100, 400} and polymer fraction in {0.2, 0.4} so that all six inputs
    (Ca, De, lambda, 2R/W, L^2, polymer fraction) vary."""
    d = sweep_sampler(k, base_seed)
    rng = np.random.default_rng(base_seed + 7919 * (k + 1))
    d["L2"] = float(rng.choice([100.0, 400.0]))
    d["polymer_fraction"] = float(rng.choice([0.2, 0.4]))
    return d


def query_triples(n: int = 32, seed: int = 4242) -> list[dict]:
    """(De, lambda, c) query triples for the Ca_cr search."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append(dict(De=float(rng.uniform(0.0, 2.0)),
                        lam=float(rng.uniform(0.5, 2.0)),
                        confinement=float(rng.uniform(0.3, 0.7)),
                        L2=100.0, polymer_fraction=0.4))
    return out


def surrogate_window_sampler(k: int, base_seed: int = 98765) -> dict:
    """Training-run sampler of the Ca_cr study window: R = 24; confinement
    c ~ U[0.45, 0.65]; De in {0, 0.5, 1, 2}; L^2 in {100, 400}; polymer
    fraction in {0.2, 0.4} (unused when De = 0); droplet phase viscoelastic.
    ``u`` ~ U[0, 1) places Ca inside the run's reachable range, and the
    viscosity ratio follows from the window's solvent rule (the caller maps
    both, since they depend on the lattice mapping)."""
    rng = np.random.default_rng(base_seed + k)
    return dict(k=k, seed=base_seed + k, R=24.0,
                confinement=float(rng.uniform(0.45, 0.65)),
                De=float(rng.choice([0.0, 0.5, 1.0, 2.0])),
                L2=float(rng.choice([100.0, 400.0])),
                polymer_fraction=float(rng.choice([0.2, 0.4])),
                u=float(rng.uniform(0.0, 1.0)), phase="DV")


def query_window(n: int = 16, seed: int = 4242) -> list[dict]:
    """Query triples (De, lambda, c) inside the study window: De ~ U[0.25, 2],
    c ~ U[0.45, 0.65], polymer fraction in {0.2, 0.4} (the viscosity ratio
    follows from it by the window's solvent rule), L^2 = 100, R = 24."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        De = float(rng.uniform(0.25, 2.0))
        c = float(rng.uniform(0.45, 0.65))
        f = float(rng.choice([0.2, 0.4]))
        out.append(dict(De=De, confinement=c, L2=100.0, polymer_fraction=f, R=24.0))
    return out


# ----------------------------------------------------------------------------
# Seeded random states for parity tests.  ``profile`` is a per-direction
# positive scale supplied by the caller (each side passes its own lattice
# table); the generator only draws uniform numbers around it.
# ----------------------------------------------------------------------------
def random_populations(shape_zyx, profile, seed, rho=(1.0, 0.04),
                       spread=0.3):
    """Two-component populations f[2][Q][nz][ny][nx] with f = rho_s(x) *
    profile[i] * (1 + spread*U(-1,1)) and rho_s(x) itself randomly mixed
    between the two component densities."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape_zyx
    q = len(profile)
    mix = rng.uniform(0.0, 1.0, size=(nz, ny, nx))
    rA = rho[0] * mix + rho[1] * (1 - mix)
    rB = rho[1] * mix + rho[0] * (1 - mix)
    prof = np.asarray(profile, dtype=np.float64).reshape(1, q, 1, 1, 1)
    base = np.stack([rA, rB])[:, None]
    noise = 1.0 + spread * rng.uniform(-1.0, 1.0, size=(2, q, nz, ny, nx))
    return np.ascontiguousarray(base * prof * noise)


def random_conformation(shape_zyx, seed, amp=0.3):
    """Symmetric positive conformation field C[6][nz][ny][nx] in the order
    (xx, yy, zz, xy, xz, yz): identity plus a random symmetric perturbation
    A A^T scaled by ``amp`` (so C stays positive definite)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape_zyx
    a = rng.uniform(-1.0, 1.0, size=(3, 3, nz, ny, nx)) * math.sqrt(amp)
    m = np.einsum("ik...,jk...->ij...", a, a)
    out = np.empty((6, nz, ny, nx))
    out[0] = 1.0 + m[0, 0]
    out[1] = 1.0 + m[1, 1]
    out[2] = 1.0 + m[2, 2]
    out[3] = m[0, 1]
    out[4] = m[0, 2]
    out[5] = m[1, 2]
    return out


def mlp_dataset(n: int, seed: int, n_in: int = 6, n_out: int = 3):
    """Random regression data (x, y, mask) for surrogate-kernel parity."""
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    y = rng.normal(size=(n, n_out)).astype(np.float32)
    y[:, 2] = (rng.uniform(size=n) < 0.5).astype(np.float32)
    mask = (rng.uniform(size=n) < 0.7).astype(np.float32)
    return x, y, mask
