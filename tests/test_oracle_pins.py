"""Pins of the FP64 oracle against facts fixed outside it: exact lattice
identities, conservation laws, Newton's third law of the Shan-Chen force,
the paper's closed-form FENE-P homogeneous-shear solution (Eqs. (6), (7)),
the exact Euler start-up of the Oldroyd-B limit, and a brute-force
node-by-node solver on tiny lattices."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as WL
from oracle import d3q19
from oracle.d3q19 import C as CV, OPP, Q, W
from oracle.scalar import scalar_step, VEL as SVEL, WT as SWT
from oracle.solver import (Oracle, Params, collide, fene_p_update, forces,
                           moments, peterlin, shan_chen_force, velocities,
                           coexistence_fractions)

# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------
def _frac_weights():
    return [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12


def test_lattice_isotropy_exact():
    w = _frac_weights()
    assert sum(w) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(w[i] * int(CV[i, a]) for i in range(Q)) == 0
        for b in range(3):
            s2 = sum(w[i] * int(CV[i, a]) * int(CV[i, b]) for i in range(Q))
            assert s2 == Fraction(d(a, b), 3)
            for c in range(3):
                s3 = sum(w[i] * int(CV[i, a] * CV[i, b] * CV[i, c]) for i in range(Q))
                assert s3 == 0
                for e in range(3):
                    s4 = sum(w[i] * int(CV[i, a] * CV[i, b] * CV[i, c] * CV[i, e])
                             for i in range(Q))
                    iso = Fraction(d(a, b) * d(c, e) + d(a, c) * d(b, e)
                                   + d(a, e) * d(b, c), 9)
                    assert s4 == iso
    for i in range(Q):
        assert tuple(CV[OPP[i]]) == tuple(-CV[i])
        assert W[i] == W[OPP[i]]


def test_lattice_matches_enumeration():
    # the brute-force solver builds its lattice by enumerating the cube
    for i in range(Q):
        assert tuple(int(v) for v in CV[i]) == SVEL[i]
        assert W[i] == SWT[i]


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.05, 1.2, size=50)
    u = rng.uniform(-0.1, 0.1, size=(3, 50))
    feq = d3q19.equilibrium(rho, u)
    assert np.allclose(feq.sum(axis=0), rho, rtol=1e-15, atol=0)
    for a in range(3):
        ja = (feq * CV[:, a, None]).sum(axis=0)
        assert np.allclose(ja, rho * u[a], rtol=0, atol=1e-16)
        for b in range(3):
            pab = (feq * (CV[:, a] * CV[:, b])[:, None]).sum(axis=0)
            want = rho * u[a] * u[b] + (rho / 3.0 if a == b else 0.0)
            assert np.allclose(pab, want, rtol=0, atol=2e-16)


# --------------------------------------------------------------------------
# Shan-Chen force
# --------------------------------------------------------------------------
def _pad_periodic_3d(a):
    return np.pad(a, 1, mode="wrap")


def test_shan_chen_newton_third_law_periodic():
    rng = np.random.default_rng(1)
    shape = (7, 6, 5)
    rA = rng.uniform(0.04, 1.0, shape)
    rB = rng.uniform(0.04, 1.0, shape)
    FA, FB = shan_chen_force(_pad_periodic_3d(rA), _pad_periodic_3d(rB), rA, rB, 0.9)
    tot = (FA + FB).sum(axis=(1, 2, 3))
    scale = np.abs(FA).sum()
    assert np.all(np.abs(tot) <= 1e-14 * scale)
    # and each component alone is not balanced (the test is not vacuous)
    assert np.abs(FA.sum(axis=(1, 2, 3))).max() > 1e-6 * scale


def test_shan_chen_uniform_and_gradient_limit():
    shape = (5, 5, 5)
    rA = np.full(shape, 0.3)
    rB = np.full(shape, 0.7)
    FA, FB = shan_chen_force(_pad_periodic_3d(rA), _pad_periodic_3d(rB), rA, rB, 0.9)
    assert np.abs(FA).max() < 1e-16 and np.abs(FB).max() < 1e-16
    # linear rho_B along x: the weights 3 w_i make sum 3 w c c = I, so the
    # force equals -G rho_A grad rho_B exactly for a linear profile
    x = np.arange(8, dtype=float)
    rB = np.broadcast_to(0.2 + 0.01 * x, (3, 3, 8)).copy()
    rA = np.full((3, 3, 8), 0.5)
    pA = np.pad(rA, 1, mode="edge")
    xp = np.arange(-1, 9, dtype=float)
    pB = np.broadcast_to(0.2 + 0.01 * xp, (5, 5, 10)).copy()
    FA, _ = shan_chen_force(pA, pB, rA, rB, 0.9)
    assert np.allclose(FA[0], -0.9 * 0.5 * 0.01, rtol=1e-13, atol=0)
    assert np.abs(FA[1]).max() < 1e-16 and np.abs(FA[2]).max() < 1e-16


def test_coexistence_fractions_mean_field():
    lo, hi = coexistence_fractions(0.9, 1.04)
    assert abs(lo + hi - 1.0) < 1e-15
    a, b = hi * 1.04, lo * 1.04
    # equal chemical potentials of the two symmetric phases
    assert abs(math.log(a / b) / 3.0 - 0.9 * (a - b)) < 1e-13
    assert abs(a - 0.9446) < 5e-4 and abs(b - 0.0954) < 5e-4


# --------------------------------------------------------------------------
# collision: per-component mass, total momentum change = total force
# --------------------------------------------------------------------------
def _random_state(shape, seed, visc=True):
    nz, ny, nx = shape
    p = WL.base_params(nx=nx, ny=ny, nz=nz, u_wall=0.01, tau=(0.8, 1.3),
                       tau_P=(20.0, 1.0) if visc else (1.0, 1.0),
                       eta_P=(0.05, 0.0) if visc else (0.0, 0.0))
    f = WL.random_populations(shape, W, seed=seed)
    C = WL.random_conformation(shape, seed=seed + 1)
    return p, f, C


def test_collision_conserves_mass_and_momentum_identity():
    shape = (6, 5, 4)
    p, f, C = _random_state(shape, 3)
    prm = Params(p)
    rho, j = moments(f)
    FA, FB = forces(rho, C, prm)
    ueqA, ueqB, u = velocities(rho, j, FA, FB, prm)
    fs = collide(f, rho, ueqA, ueqB, prm)
    rho2, j2 = moments(fs)
    assert np.allclose(rho2, rho, rtol=1e-15, atol=0)
    dj = (j2[0] + j2[1]) - (j[0] + j[1])
    assert np.allclose(dj, FA + FB, rtol=0, atol=1e-15)
    # half-force physical velocity
    assert np.allclose(u * (rho[0] + rho[1]), j[0] + j[1] + 0.5 * (FA + FB),
                       rtol=1e-14, atol=1e-17)


# --------------------------------------------------------------------------
# whole step: brute force, mass conservation with moving walls
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape_xyz", [(3, 4, 5), (6, 5, 7)])
@pytest.mark.parametrize("visc", [True, False])
@pytest.mark.parametrize("trt", [False, True])
def test_vectorised_matches_brute_force(shape_xyz, visc, trt):
    nx, ny, nz = shape_xyz
    p, f, C = _random_state((nz, ny, nx), 11, visc)
    if trt:
        p = dict(p, tau_minus=(0.7, 1.9))
    o = Oracle(p, f=f, C=C)
    prm = Params(p)
    fs, Cs = f.copy(), C.copy()
    for _ in range(3):
        o.step()
        fs, Cs = scalar_step(fs, Cs, prm)
        fs, Cs = np.array(fs), np.array(Cs)
        assert np.abs(o.f - fs).max() <= 1e-14 * np.abs(fs).max()
        assert np.abs(o.C - Cs).max() <= 1e-14 * np.abs(Cs).max()
    if visc:
        assert np.abs(o.C - C).max() > 1e-3     # the polymer part did move


def test_mass_conserved_with_moving_walls():
    shape = (8, 6, 7)
    p, f, C = _random_state(shape, 5)
    o = Oracle(p, f=f, C=C)
    m0 = o.f.sum(axis=(1, 2, 3, 4))
    o.step(50)
    m1 = o.f.sum(axis=(1, 2, 3, 4))
    assert np.all(np.abs(m1 - m0) <= 1e-13 * m0)
    assert o.status == 0


# --------------------------------------------------------------------------
# FENE-P: paper Eqs. (6) and (7) (homogeneous shear u_x = gamma_dot z)
# --------------------------------------------------------------------------
def _shear_padded(shape, gdot):
    nz, ny, nx = shape
    up = np.zeros((3, nz + 2, ny + 2, nx + 2))
    zz = np.arange(-1, nz + 1, dtype=float)
    up[0] = gdot * zz[:, None, None]
    return up, up[:, 1:-1, 1:-1, 1:-1].copy()


def _paper_eq6_eq7(wi, L2):
    arg = (wi * L2 / 4.0) * (L2 / 6.0) ** -1.5
    sh = math.sinh(math.asinh(arg) / 3.0)
    s = 2.0 * math.sqrt(L2 / 6.0) * sh          # f C_xz, Eq. (6) / (eta_P/tau_P)
    n1 = 8.0 * (L2 / 6.0) * sh * sh             # f (C_xx - C_yy), Eq. (7)
    return s, n1


@pytest.mark.parametrize("wi,L2", [(0.5, 100.0), (1.0, 100.0), (2.0, 100.0),
                                   (1.0, 400.0), (5.0, 100.0)])
def test_fene_p_homogeneous_shear_matches_paper(wi, L2):
    shape = (3, 3, 3)
    tau_P = 10.0
    gdot = wi / tau_P
    p = WL.base_params(nx=3, ny=3, nz=3, tau_P=(tau_P, 1.0), eta_P=(0.1, 0.0),
                       L2=(L2, L2))
    prm = Params(p)
    up, u = _shear_padded(shape, gdot)
    C = np.zeros((6,) + shape)
    C[0] = C[1] = C[2] = 1.0
    for _ in range(4000):
        C = fene_p_update(C, u, prm, u_p=up)
    f = peterlin(C, L2)
    s, n1 = _paper_eq6_eq7(wi, L2)
    assert np.allclose(f * C[4], s, rtol=1e-12, atol=0)
    assert np.allclose(f * (C[0] - C[1]), n1, rtol=1e-12, atol=0)
    assert np.allclose(C[1], C[2], rtol=1e-13) and np.allclose(C[1], 1.0 / f, rtol=1e-12)
    assert np.abs(C[3]).max() < 1e-15 and np.abs(C[5]).max() < 1e-15


def test_fene_p_peterlin_consistency_at_wi_1():
    # Wi = 1, L^2 = 100: f^2 (f - 1) = 2 Wi^2 / L^2 (consistency of Eq. (6)
    # with the Peterlin factor); f = 1.019251615479
    s, _ = _paper_eq6_eq7(1.0, 100.0)
    f = 1.0 / s
    assert abs(f * f * (f - 1.0) - 0.02) < 1e-14
    assert abs(f - 1.019251615479) < 1e-11


def test_oldroyd_b_euler_startup_exact():
    tau_P, wi = 25.0, 1.3
    gdot = wi / tau_P
    shape = (3, 3, 3)
    p = WL.base_params(nx=3, ny=3, nz=3, tau_P=(tau_P, 1.0), eta_P=(0.1, 0.0),
                       L2=(1e12, 1e12))
    prm = Params(p)
    up, u = _shear_padded(shape, gdot)
    C = np.zeros((6,) + shape)
    C[0] = C[1] = C[2] = 1.0
    for n in range(1, 60):
        C = fene_p_update(C, u, prm, u_p=up)
        want_xz = wi * (1.0 - (1.0 - 1.0 / tau_P) ** n)
        assert np.allclose(C[4], want_xz, rtol=1e-10, atol=0)
        assert np.allclose(C[2], 1.0, rtol=0, atol=1e-10)


def test_fene_p_upwind_advection_of_a_step():
    # pure advection at |u| = 0.5 along +x of a step in C_xx: first-order
    # upwind moves the profile as the exact linear recursion
    # c_new(x) = c(x) - u (c(x) - c(x-1)) (no shear, relaxation switched off
    # by L^2 huge and tau_P huge)
    nz, ny, nx = 3, 3, 12
    p = WL.base_params(nx=nx, ny=ny, nz=nz, tau_P=(1e30, 1.0), eta_P=(0.1, 0.0),
                       L2=(1e30, 1e30))
    prm = Params(p)
    u = np.zeros((3, nz, ny, nx))
    u[0] = 0.5
    up = np.pad(u, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap")
    C = np.zeros((6, nz, ny, nx))
    C[0] = 1.0 + (np.arange(nx) >= 6)[None, None, :]
    C[1] = C[2] = 1.0
    Cn = fene_p_update(C, u, prm, u_p=up)
    c = C[0, 0, 0]
    want = c - 0.5 * (c - np.roll(c, 1))
    assert np.allclose(Cn[0, 1, 1], want, rtol=0, atol=1e-15)
    u[0] = -0.5
    up = np.pad(u, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap")
    Cn = fene_p_update(C, u, prm, u_p=up)
    want = c - (-0.5) * (np.roll(c, -1) - c)
    assert np.allclose(Cn[0, 1, 1], want, rtol=0, atol=1e-15)


def test_splitmix64_published_words():
    """The initial-noise generator is SplitMix64 (Steele, Lea and Flood 2014):
    its first five words for seed 0 are the published ones, and the noise
    factors are 1 + a u with u uniform in [-1, 1)."""
    import numpy as np
    from oracle.solver import Params, init_noise_factors, splitmix64
    import workloads as WL
    w = splitmix64(0, np.arange(5))
    assert [int(v) for v in w] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                                   0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    d = dict(WL.base_params(nx=40, ny=30, nz=20, radius=5.0), seed=2024, init_noise=0.01)
    fac = init_noise_factors(Params(d))
    u = (fac - 1.0) / 0.01
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.02 and abs(u.var() - 1.0 / 3.0) < 0.02
    # the two components draw different words; another seed, another field
    assert not np.array_equal(fac[0], fac[1])
    d2 = dict(d, seed=2025)
    assert not np.array_equal(init_noise_factors(Params(d2)), fac)
    # no noise: every factor is exactly one
    assert np.all(init_noise_factors(Params(dict(d, init_noise=0.0))) == 1.0)
