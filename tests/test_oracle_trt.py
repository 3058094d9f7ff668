"""Pins of the oracle's two-relaxation-time collision (a model variant: the
paper's scheme is BGK).  Each check is fixed by the definition of the
collision or by a closed-form solution, not by the oracle's own formula:
  * equal rates reduce it to BGK;
  * every moment of f that is even under c -> -c relaxes towards its
    equilibrium value by the factor (1 - 1/tau^+), every odd one by
    (1 - 1/tau^-); mass and the momentum change follow;
  * with the velocity shift taken at tau^-, a collision conserves the total
    momentum up to the forces;
  * plane Couette flow is linear for any pair of rates, and force-driven
    channel flow between half-way bounce-back walls is the parabola
    g/(2 nu) [(z + 1/2)(W - 1/2 - z) + (16 Lambda - 3)/12] with
    nu = (tau^+ - 1/2)/3 and Lambda = (tau^+ - 1/2)(tau^- - 1/2): exact at
    Lambda = 3/16, with the Lambda-dependent wall slip otherwise (Ginzburg
    and d'Humieres, Phys. Rev. E 68, 066614 (2003))."""
import numpy as np
import pytest

import workloads as WL
from oracle import d3q19
from oracle.d3q19 import C as CV, OPP, Q, W
from oracle.solver import Oracle, collide_trt


def _random_state(rng, shape=(4, 3, 5)):
    rho = 1.0 + 0.3 * rng.random(shape)
    u = 0.05 * (rng.random((3,) + shape) - 0.5)
    feq = d3q19.equilibrium(rho, u)
    f = feq * (1.0 + 0.2 * (rng.random((Q,) + shape) - 0.5))
    return f, feq


def test_equal_rates_are_bgk():
    rng = np.random.default_rng(11)
    f, feq = _random_state(rng)
    for tau in (0.6, 1.0, 1.7):
        bgk = f - (f - feq) / tau
        assert np.allclose(collide_trt(f, feq, tau, tau), bgk, rtol=0, atol=1e-15)


def test_even_and_odd_moments_relax_at_their_own_rates():
    rng = np.random.default_rng(12)
    f, feq = _random_state(rng)
    tp, tm = 1.3, 0.7
    out = collide_trt(f, feq, tp, tm)
    cx, cy, cz = (CV[:, k].astype(float) for k in range(3))
    even = [np.ones(Q), cx * cx, cy * cy, cz * cz, cx * cy, cx * cz, cy * cz,
            cx * cx * cy * cy, cy * cy * cz * cz, cx * cx * cz * cz]
    odd = [cx, cy, cz, cx * cy * cy, cx * cz * cz, cy * cx * cx, cy * cz * cz,
           cz * cx * cx, cz * cy * cy]
    for v in even + odd:
        assert np.array_equal(v, v[OPP]) or np.array_equal(v, -v[OPP])
    mom = lambda g, v: np.tensordot(v, g, axes=(0, 0))
    for vs, tau in ((even, tp), (odd, tm)):
        for v in vs:
            want = (1.0 - 1.0 / tau) * (mom(f, v) - mom(feq, v))
            assert np.allclose(mom(out, v) - mom(feq, v), want, rtol=0, atol=1e-14)


def test_collision_conserves_total_momentum_up_to_the_forces():
    """A random two-component state with Shan-Chen forces: sum over both
    components of the post-collision momentum equals the pre-collision
    momentum plus the total force, for unequal tau^- of the components."""
    from oracle.solver import collide
    rng = np.random.default_rng(13)
    p = WL.base_params(nx=6, ny=5, nz=4, radius=2.0, tau=(0.9, 1.4), tau_minus=(0.75, 1.1))
    o = Oracle(p)
    o.f = o.f * (1.0 + 0.05 * (rng.random(o.f.shape) - 0.5))
    rho, j, FA, FB, ueqA, ueqB, _u = o.flow()
    fs = collide(o.f, rho, ueqA, ueqB, o.prm)
    jn = np.einsum("sq...,qa->sa...", fs, CV.astype(float))
    assert np.allclose(jn.sum(axis=0), j.sum(axis=0) + FA + FB, rtol=0, atol=1e-14)
    # each component's momentum moves towards rho_s u^eq_s at 1/tau^-_s
    for s, ueq in ((0, ueqA), (1, ueqB)):
        tm = o.prm.tau_minus[s]
        assert np.allclose(jn[s], j[s] + (rho[s] * ueq - j[s]) / tm, rtol=0, atol=1e-14)


def _channel(tp, tm, nz=8, g=0.0, uw=0.0, steps=1500):
    p = WL.base_params(nx=3, ny=3, nz=nz, u_wall=uw, radius=0.0, rho_major=1.0, rho_minor=1.0,
                       G=0.0, tau=(tp, tp), tau_minus=(tm, tm))
    p["body_accel"] = (g, 0.0, 0.0)
    o = Oracle(p)
    o.step(steps)
    u = o.velocity()
    return u, np.arange(nz)


@pytest.mark.parametrize("tp,tm", [(1.4, 0.7), (0.8, 1.9)])
def test_couette_is_linear_for_any_rates(tp, tm):
    nz, uw = 8, 0.004
    u, z = _channel(tp, tm, nz=nz, uw=uw, steps=1200)
    want = uw * (2 * z + 1 - nz) / nz
    for y in range(3):
        for x in range(3):
            assert np.abs(u[0, :, y, x] - want).max() < 1e-12 * uw
    assert np.abs(u[1]).max() < 1e-12 * uw and np.abs(u[2]).max() < 1e-12 * uw


@pytest.mark.parametrize("tp,tm", [(2.0, 0.625), (1.0, 0.875), (2.0, 2.0), (1.0, 1.0)])
def test_channel_flow_wall_slip_follows_lambda(tp, tm):
    """(2.0, 0.625) and (1.0, 0.875) sit at Lambda = 3/16 (the parabola
    through the half-way walls exactly); the BGK pairs have Lambda = 2.25
    and 1/4 and a uniform slip of (16 Lambda - 3)/12 in units of g/(2 nu)."""
    nz, g = 8, 1e-5
    u, z = _channel(tp, tm, nz=nz, g=g)
    nu = (tp - 0.5) / 3.0
    lam = (tp - 0.5) * (tm - 0.5)
    want = g / (2 * nu) * ((z + 0.5) * (nz - 0.5 - z) + (16 * lam - 3) / 12)
    scale = g / (2 * nu) * (nz / 2) ** 2
    assert np.abs(u[0, :, 1, 1] - want).max() < 1e-10 * scale
    if lam != 0.1875:
        exact_walls = g / (2 * nu) * (z + 0.5) * (nz - 0.5 - z)
        assert np.abs(u[0, :, 1, 1] - exact_walls).max() > 1e-3 * scale
