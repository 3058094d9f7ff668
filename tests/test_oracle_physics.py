"""Physics pins of the FP64 oracle: plane Couette flow between the moving
walls (Section 3 set-up), the Laplace law for static droplets, symmetries
of a droplet in confined shear, and the observables and component counter on
synthetic shapes whose answers are known in closed form."""
import math

import numpy as np
import pytest

import workloads as WL
from oracle.components import component_sizes
from oracle.d3q19 import Q, W
from oracle.observables import observe
from oracle.solver import Oracle


def test_couette_linear_profile():
    """Uniform mixture between walls at +-U_w: the steady profile is the
    linear shear u_x(z) = U_w (2z + 1 - nz)/nz through the wall planes at
    z = -1/2 and nz - 1/2 (gamma_dot = 2U_w/W, W = nz)."""
    nz = 16
    p = WL.base_params(nx=4, ny=4, nz=nz, radius=0.0, u_wall=0.005)
    o = Oracle(p)
    o.step(2000)
    u = o.velocity()
    z = np.arange(nz)
    want = 0.005 * (2 * z + 1 - nz) / nz
    for y in range(4):
        for x in range(4):
            err = np.sqrt(((u[0, :, y, x] - want) ** 2).sum() / (want ** 2).sum())
            assert err < 1e-9
    assert np.abs(u[1]).max() < 1e-14 and np.abs(u[2]).max() < 1e-14


def test_couette_with_polymer_homogeneous_shear():
    """Polymer everywhere (the polymer phase is the majority of the whole box,
    so its indicator is 1): the flow stays linear and the conformation tensor
    reaches the homogeneous-shear state of Eqs. (6)-(7) at Wi = gamma_dot
    tau_P (the wall ghosts extrapolate u linearly, so grad u is uniform)."""
    nz, uw, tau_P, L2 = 16, 0.005, 400.0, 100.0
    p = WL.base_params(nx=3, ny=3, nz=nz, radius=0.0, u_wall=uw,
                       tau_P=(1.0, tau_P), eta_P=(0.0, 0.02), L2=(L2, L2))
    o = Oracle(p)
    o.step(6000)
    gdot = 2 * uw / nz
    wi = gdot * tau_P
    arg = (wi * L2 / 4.0) * (L2 / 6.0) ** -1.5
    s = 2.0 * math.sqrt(L2 / 6.0) * math.sinh(math.asinh(arg) / 3.0)
    C = o.C
    f = (L2 - 3.0) / (L2 - C[0] - C[1] - C[2])
    assert np.allclose(f * C[4], s, rtol=1e-6)
    u = o.velocity()
    z = np.arange(nz)
    want = uw * (2 * z + 1 - nz) / nz
    err = np.sqrt(((u[0, :, 1, 1] - want) ** 2).sum() / (want ** 2).sum())
    assert err < 1e-6


def _cylinder_laplace(R, n=40, steps=2000):
    """Static cylindrical droplet (axis along y, ny = 1 so the lattice acts as
    its 2D projection).  Returns (pressure jump, effective radius) with the
    Shan-Chen bulk pressure P = (rho_A + rho_B)/3 + G rho_A rho_B."""
    p = WL.base_params(nx=n, ny=1, nz=n, radius=float(R), u_wall=0.0)
    o = Oracle(p)
    o.step(steps)
    rho = o.density()
    rA, rB = rho[0, :, 0, :], rho[1, :, 0, :]
    P = (rA + rB) / 3.0 + 0.9 * rA * rB
    c = n // 2
    dp = P[c - 1:c + 1, c - 1:c + 1].mean() - P[0:2, 0:2].mean()
    ain, aout = rA[c - 1:c + 1, c - 1:c + 1].mean(), rA[0:2, 0:2].mean()
    area = ((rA - aout) / (ain - aout)).sum()
    return dp, math.sqrt(area / math.pi)


def test_laplace_law_cylinders():
    """Laplace: dp = sigma / R for a cylinder, so dp * R_eff is the same for
    every radius (4 % for a diffuse interface of ~3 nodes at R = 6..10)."""
    vals = []
    for R in (6.0, 8.0, 10.0):
        dp, reff = _cylinder_laplace(R)
        assert dp > 0.0
        vals.append(dp * reff)
    vals = np.array(vals)
    assert (vals.max() - vals.min()) / vals.mean() < 0.04
    # separated phases: minority density inside the droplet is small
    assert 0.1 < vals.mean() < 0.3


def test_droplet_in_shear_symmetries():
    """A centred droplet in plane Couette flow is invariant under the 180
    degree rotation about the y axis through the centre and under the
    reflection y -> -y; the centroid stays at the centre."""
    p = WL.base_params(nx=16, ny=12, nz=16, radius=4.0, u_wall=0.01)
    o = Oracle(p)
    o.step(150)
    rho = o.density()
    rot = rho[:, ::-1, :, ::-1]          # (x, z) -> (-x, -z) about the centre
    assert np.abs(rho - rot).max() < 1e-12
    assert np.abs(rho - rho[:, :, ::-1, :]).max() < 1e-12
    u = o.velocity()
    assert np.abs(u[0] + u[0][::-1, :, ::-1]).max() < 1e-12
    assert np.abs(u[1].sum()) < 1e-12
    obs = observe(o.f, o.C)
    assert np.allclose(obs["centroid"], (7.5, 5.5, 7.5), rtol=0, atol=1e-10)
    assert obs["D"] > 1e-4                          # it does deform
    assert 0.0 < obs["theta_deg"] < 90.0


# --------------------------------------------------------------------------
# observables on synthetic fields
# --------------------------------------------------------------------------
def _state_from_mask(mask):
    """Populations whose phase field is +1 on mask nodes and -1 elsewhere."""
    nz, ny, nx = mask.shape
    rhoA = np.where(mask, 1.0, 0.0)
    rhoB = np.where(mask, 0.0, 1.0)
    f = np.zeros((2, Q, nz, ny, nx))
    for i in range(Q):
        f[0, i] = W[i] * rhoA
        f[1, i] = W[i] * rhoB
    C = np.zeros((6, nz, ny, nx))
    C[0] = C[1] = C[2] = 1.0
    return f, C


def test_observables_rectangle():
    nz, ny, nx = 20, 3, 30
    mask = np.zeros((nz, ny, nx), bool)
    a, b = 11, 5                       # extent along x and along z
    mask[6:6 + b, :, 4:4 + a] = True
    f, C = _state_from_mask(mask)
    obs = observe(f, C)
    Ixx = ny * b * a * (a * a - 1) / 12.0
    Izz = ny * a * b * (b * b - 1) / 12.0
    assert np.isclose(obs["inertia"][0], Ixx, rtol=1e-13)
    assert np.isclose(obs["inertia"][2], Izz, rtol=1e-13)
    assert abs(obs["inertia"][1]) < 1e-10
    D = (math.sqrt(Ixx) - math.sqrt(Izz)) / (math.sqrt(Ixx) + math.sqrt(Izz))
    assert np.isclose(obs["D"], D, rtol=1e-13)
    assert abs(obs["theta_deg"]) < 1e-12
    assert obs["Lp"] == a
    assert np.allclose(obs["centroid"], (4 + (a - 1) / 2, 1.0, 6 + (b - 1) / 2))
    assert np.allclose(obs["mass"], (a * b * ny, nz * ny * nx - a * b * ny),
                       rtol=1e-14)


def test_observables_tilted_segment():
    # nodes on the diagonal x - x0 = z - z0: a line at 45 degrees, D = 1
    nz, ny, nx = 20, 1, 20
    mask = np.zeros((nz, ny, nx), bool)
    for k in range(9):
        mask[5 + k, 0, 3 + k] = True
    f, C = _state_from_mask(mask)
    obs = observe(f, C)
    assert abs(obs["theta_deg"] - 45.0) < 1e-12
    assert abs(obs["D"] - 1.0) < 1e-12
    assert obs["Lp"] == 9


def test_component_sizes_synthetic():
    m = np.zeros((6, 5, 10), bool)
    m[1:3, 1:3, 1:3] = True                 # block of 8
    m[4, 2, 6] = True                       # isolated node
    assert component_sizes(m) == [8, 1]
    m2 = np.zeros((6, 5, 10), bool)
    m2[2, 2, 0] = m2[2, 2, 9] = True        # joined across the periodic x seam
    m2[2, 0, 4] = m2[2, 4, 4] = True        # joined across the periodic y seam
    m2[0, 1, 1] = m2[5, 1, 1] = True        # NOT joined across the z walls
    assert component_sizes(m2) == [2, 2, 1, 1]
    m3 = np.zeros((4, 4, 4), bool)
    m3[1, 1, 1] = m3[2, 2, 2] = True        # corner contact only: 2 components
    assert component_sizes(m3) == [1, 1]
