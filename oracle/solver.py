"""Array-at-a-time FP64 oracle of one hybrid LB/FD step (TEST INFRASTRUCTURE).

Continuum model (paper Section 2): in each phase the Navier-Stokes equation
with the polymer body force (eta_P/tau_P) div[f(r_P) C] (Eqs. (1) and (3)),
and the FENE-P law dC/dt + (u.grad)C = C.grad(u) + grad(u)^T.C - (f C - I)/tau_P
(Eqs. (2) and (4)) with the Peterlin factor f = (L^2-3)/(L^2 - tr C) (defined
below Eq. (2)).  Immiscibility comes from the Shan-Chen interaction between
the two lattice-Boltzmann components (Section 2).  The viscosity ratio is set
on total viscosity and polymer lives in one phase only (Section 2, the
paragraph that introduces MV and DV).  Walls move at +-U_w along x, periodic
in x and y, sphere at mid-gap (Section 3, set-up paragraph).

Discrete readings (the paper defers the discretisation to its methods paper):
  * D3Q19, BGK, one relaxation time per component (oracle.d3q19).
  * Shan-Chen force with psi = rho and interaction weights 3 w_i:
        F^SC_s(x) = -G rho_s(x) sum_{i>0} 3 w_i rho_sbar(x + c_i) c_i.
  * Polymer stress T = chi (eta_P/tau_P) (f C - I), chi the clamped rescaled
    mass fraction of the polymer phase's component; force
    F^P_a = sum_b [T_ab(x+e_b) - T_ab(x-e_b)]/2, split over the components
    by mass fraction.
  * Shan-Chen velocity-shift forcing: u' = sum_s(j_s/tau_s)/sum_s(rho_s/tau_s),
    u^eq_s = u' + tau_s F_s/rho_s; physical u = (sum_s j_s + sum_s F_s/2)/rho.
  * Optional two-relaxation-time collision (a model variant beyond the
    paper's BGK): the parts of f symmetric and antisymmetric under c -> -c
    relax at 1/tau and 1/tau^-.  Momentum is the antisymmetric moment, so
    the velocity shift takes tau^- wherever BGK has tau: the collision
    changes j_s by (rho_s u^eq_s - j_s)/tau^-_s, which conserves the total
    momentum up to the forces.  tau^- = tau is BGK.
  * FENE-P by explicit Euler with dt = 1: centred grad u, first-order upwind
    advection; C^{n+1} uses u^n and C^n; F^P uses C^n.
  * Ghosts: rho mirror in z, C zero-gradient in z, u extrapolated linearly
    through the wall velocity; periodic in x and y.
  * Half-way bounce-back on moving walls (walls half a link outside z=0 and
    z=nz-1): f_opp(i)(x) = f*_i(x) - 6 w_i rho_s(x) c_i.u_wall.
  * Initial state: f = w_i rho_s, u = 0, C = I; sphere |x-c|^2 < R^2 strict.
"""
from __future__ import annotations

import math

import numpy as np

from . import d3q19
from .d3q19 import C as CV, OPP, Q, W

STATUS_NAN = 1
STATUS_FENE = 2

# component order of the symmetric conformation tensor
_SYM = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3,
        (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}


def coexistence_fractions(G: float, rho_tot: float):
    """Mean-field coexistence mass fractions (minority, majority) of the
    symmetric two-component Shan-Chen mixture with psi = rho and unit-sum
    interaction weights: equal chemical potentials of the two symmetric
    phases give atanh(m) = (3/2) G rho_tot m for the order parameter m.
    Solved by bisection.  Without demixing, returns (None, None)."""
    k = 1.5 * G * rho_tot
    if k <= 1.0:
        return None, None
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= 0.0 or mid >= 1.0:
            break
        if math.atanh(mid) - k * mid > 0.0:
            hi = mid
        else:
            lo = mid
    m = 0.5 * (lo + hi)
    return 0.5 * (1.0 - m), 0.5 * (1.0 + m)


class Params:
    """Lattice parameters of one run (plain attributes, FP64)."""

    def __init__(self, d: dict):
        self.nx, self.ny, self.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
        self.u_wall = float(d["u_wall"])
        self.radius = float(d["radius"])
        cx, cy, cz = float(d["cx"]), float(d["cy"]), float(d["cz"])
        if cx < 0:
            cx, cy, cz = (self.nx - 1) / 2, (self.ny - 1) / 2, (self.nz - 1) / 2
        self.centre = (cx, cy, cz)
        self.rho_major = float(d["rho_major"])
        self.rho_minor = float(d["rho_minor"])
        self.G = float(d["G"])
        self.tau = tuple(float(t) for t in d["tau"])
        self.tau_P = tuple(float(t) for t in d["tau_P"])
        self.eta_P = tuple(float(t) for t in d["eta_P"])
        self.L2 = tuple(float(t) for t in d["L2"])
        visc = [p for p in (0, 1) if self.eta_P[p] > 0.0]
        if len(visc) > 1:
            raise ValueError("at most one viscoelastic phase")
        self.phase = visc[0] if visc else None
        lo, hi = float(d.get("chi_lo", 0.0)), float(d.get("chi_hi", 0.0))
        if lo == 0.0 and hi == 0.0:
            rt = self.rho_major + self.rho_minor
            lo, hi = coexistence_fractions(self.G, rt)
            if lo is None:
                lo, hi = self.rho_minor / rt, self.rho_major / rt
        self.chi_lo, self.chi_hi = lo, hi
        self.seed = int(d.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
        self.init_noise = float(d.get("init_noise", 0.0))
        # antisymmetric relaxation times (0 or absent: tau, i.e. BGK)
        tm = d.get("tau_minus") or (0.0, 0.0)
        self.tau_minus = tuple(float(t) if float(t) > 0.0 else self.tau[s]
                               for s, t in enumerate(tm))
        # uniform acceleration g, F_s += rho_s g (closed-form channel tests)
        self.body_accel = tuple(float(v) for v in d.get("body_accel", (0.0, 0.0, 0.0)))


def splitmix64(seed: int, k):
    """Words k (uint64 array) of SplitMix64 with the given seed (Steele, Lea
    and Flood, OOPSLA 2014): the finaliser applied to seed + (k + 1) * gamma,
    gamma = 0x9e3779b97f4a7c15, all modulo 2^64."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(k, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9e3779b97f4a7c15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xbf58476d1ce4e5b9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94d049bb133111eb)
        return z ^ (z >> np.uint64(31))


def init_noise_factors(p):
    """1 + a u per component and node (shape (2, nz, ny, nx)), u in [-1, 1)
    from word 2 n + s of SplitMix64 (n the node index, x fastest): the
    optional seeded perturbation of the initial densities."""
    n = np.arange(p.nx * p.ny * p.nz, dtype=np.uint64).reshape(p.nz, p.ny, p.nx)
    out = np.empty((2, p.nz, p.ny, p.nx))
    for s in (0, 1):
        w = splitmix64(p.seed, np.uint64(2) * n + np.uint64(s))
        u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
        out[s] = 1.0 + p.init_noise * u
    return out


# --------------------------------------------------------------------------
# ghost layers (one node wide): periodic in x and y, z rule given per field
# --------------------------------------------------------------------------
def _pad_xy_periodic(a):
    """(..., nz, ny, nx) -> (..., nz, ny+2, nx+2), periodic copies."""
    nd = a.ndim
    width = [(0, 0)] * (nd - 2) + [(1, 1), (1, 1)]
    return np.pad(a, width, mode="wrap")


def pad_mirror_z(a):
    """Ghost planes equal to the boundary planes (rho mirror, C zero
    gradient)."""
    p = _pad_xy_periodic(a)
    nd = p.ndim
    width = [(0, 0)] * (nd - 3) + [(1, 1), (0, 0), (0, 0)]
    return np.pad(p, width, mode="edge")


def pad_velocity(u, u_wall):
    """u (3, nz, ny, nx): ghost planes u(-1) = 2 u_bot - u(0),
    u(nz) = 2 u_top - u(nz-1) with u_bot = (-U_w,0,0), u_top = (+U_w,0,0)."""
    p = _pad_xy_periodic(u)
    nz = u.shape[1]
    out = np.empty((3, nz + 2) + p.shape[2:])
    out[:, 1:-1] = p
    wall_bot = np.array([-u_wall, 0.0, 0.0]).reshape(3, 1, 1)
    wall_top = np.array([u_wall, 0.0, 0.0]).reshape(3, 1, 1)
    out[:, 0] = 2.0 * wall_bot - p[:, 0]
    out[:, -1] = 2.0 * wall_top - p[:, -1]
    return out


def _shift(p, d, shape):
    """View of a padded array at offset d = (dx, dy, dz) from each node."""
    nz, ny, nx = shape
    dx, dy, dz = d
    return p[..., 1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


_E = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
_NEG = ((-1, 0, 0), (0, -1, 0), (0, 0, -1))


# --------------------------------------------------------------------------
# the pieces of one step
# --------------------------------------------------------------------------
def moments(f):
    """rho_s = sum_i f_si, j_s = sum_i f_si c_i.  f (2, Q, nz, ny, nx)."""
    rho = f.sum(axis=1)
    j = np.zeros((2, 3) + f.shape[2:])
    for i in range(Q):
        for a in range(3):
            if CV[i, a] != 0:
                j[:, a] += CV[i, a] * f[:, i]
    return rho, j


def shan_chen_force(rhoA_p, rhoB_p, rhoA, rhoB, G):
    """F^SC_A = -G rho_A(x) sum_i 3 w_i rho_B(x+c_i) c_i and the mirror
    expression for B, from ghost-padded densities."""
    shape = rhoA.shape
    sA = np.zeros((3,) + shape)
    sB = np.zeros((3,) + shape)
    for i in range(1, Q):
        wt = 3.0 * W[i]
        c = tuple(int(v) for v in CV[i])
        nbB = _shift(rhoB_p, c, shape)
        nbA = _shift(rhoA_p, c, shape)
        for a in range(3):
            if c[a] != 0:
                sA[a] += (wt * c[a]) * nbB
                sB[a] += (wt * c[a]) * nbA
    return -G * rhoA * sA, -G * rhoB * sB


def peterlin(C, L2):
    """f(r_P) = (L^2 - 3)/(L^2 - tr C) with r_P^2 = tr C (below Eq. (2))."""
    tr = C[0] + C[1] + C[2]
    return (L2 - 3.0) / (L2 - tr)


def polymer_stress(C, rhoA, rhoB, prm: Params):
    """T_kl = chi (eta_P/tau_P) (f C_kl - delta_kl) for the six components;
    works on padded or unpadded arrays alike."""
    p = prm.phase
    rho_p = rhoA if p == 0 else rhoB
    xp = rho_p / (rhoA + rhoB)
    chi = np.clip((xp - prm.chi_lo) / (prm.chi_hi - prm.chi_lo), 0.0, 1.0)
    fP = peterlin(C, prm.L2[p])
    coef = chi * (prm.eta_P[p] / prm.tau_P[p])
    T = np.empty_like(C)
    for k in range(6):
        delta = 1.0 if k < 3 else 0.0
        T[k] = coef * (fP * C[k] - delta)
    return T


def polymer_force(T_p, shape):
    """F^P_a = sum_b [T_ab(x + e_b) - T_ab(x - e_b)] / 2 (centred divergence
    of the stress of Eqs. (1)/(3))."""
    F = np.zeros((3,) + shape)
    for a in range(3):
        for b in range(3):
            k = _SYM[(a, b)]
            F[a] += 0.5 * (_shift(T_p[k], _E[b], shape)
                           - _shift(T_p[k], _NEG[b], shape))
    return F


def forces(rho, C, prm: Params):
    """Total force on each component, F_s = F^SC_s + (rho_s/rho) F^P
    (+ rho_s g with the optional uniform acceleration g)."""
    rhoA, rhoB = rho[0], rho[1]
    shape = rhoA.shape
    rhoA_p, rhoB_p = pad_mirror_z(rhoA), pad_mirror_z(rhoB)
    FA, FB = shan_chen_force(rhoA_p, rhoB_p, rhoA, rhoB, prm.G)
    if any(prm.body_accel):
        g = np.array(prm.body_accel).reshape(3, 1, 1, 1)
        FA = FA + rhoA * g
        FB = FB + rhoB * g
    if prm.phase is not None:
        T_p = polymer_stress(pad_mirror_z(C), rhoA_p, rhoB_p, prm)
        FP = polymer_force(T_p, shape)
        rtot = rhoA + rhoB
        FA = FA + (rhoA / rtot) * FP
        FB = FB + (rhoB / rtot) * FP
    return FA, FB


def velocities(rho, j, FA, FB, prm: Params):
    """Shan-Chen common velocity u', per-component equilibrium velocities
    u^eq_s = u' + tau_s F_s/rho_s, and the physical velocity
    u = (j_A + j_B + (F_A + F_B)/2)/rho.  tau_s is the relaxation time of
    the momentum: tau^-_s (equal to tau_s under BGK)."""
    tA, tB = prm.tau_minus
    rhoA, rhoB = rho[0], rho[1]
    up = (j[0] / tA + j[1] / tB) / (rhoA / tA + rhoB / tB)
    ueqA = up + tA * FA / rhoA
    ueqB = up + tB * FB / rhoB
    u = (j[0] + j[1] + 0.5 * (FA + FB)) / (rhoA + rhoB)
    return ueqA, ueqB, u


def collide(f, rho, ueqA, ueqB, prm: Params):
    """BGK: f*_si = f_si - (f_si - f^eq_i(rho_s, u^eq_s))/tau_s; a component
    with tau^-_s != tau_s takes the two-relaxation-time collision."""
    out = np.empty_like(f)
    for s, ueq in ((0, ueqA), (1, ueqB)):
        feq = d3q19.equilibrium(rho[s], ueq)
        if prm.tau_minus[s] == prm.tau[s]:
            out[s] = f[s] - (f[s] - feq) / prm.tau[s]
        else:
            out[s] = collide_trt(f[s], feq, prm.tau[s], prm.tau_minus[s])
    return out


def collide_trt(f, feq, tau_plus, tau_minus):
    """Two-relaxation-time collision of one component: with
    f^+-_i = (f_i +- f_opp(i))/2 and the same split of f^eq,
    f*_i = f_i - (f^+_i - f^eq+_i)/tau^+ - (f^-_i - f^eq-_i)/tau^-."""
    fo, eo = f[OPP], feq[OPP]
    fp, fm = 0.5 * (f + fo), 0.5 * (f - fo)
    ep, em = 0.5 * (feq + eo), 0.5 * (feq - eo)
    return f - (fp - ep) / tau_plus - (fm - em) / tau_minus


def fene_p_update(C, u, prm: Params, u_p=None):
    """Explicit Euler step of Eq. (2)/(4) with dt = 1:
    C^{n+1} = C - A + S - (f C - I)/tau_P, where
      G_ab = d_a u_b = [u_b(x+e_a) - u_b(x-e_a)]/2,
      A_kl = sum_a max(u_a,0)(C_kl(x)-C_kl(x-e_a))
                 + min(u_a,0)(C_kl(x+e_a)-C_kl(x))   (first-order upwind),
      S_kl = sum_m C_km G_ml + G_mk C_ml.
    ``u_p`` may supply a ghost-padded velocity (tests use it to impose a
    prescribed flow); by default the wall rule of pad_velocity applies."""
    p = prm.phase
    shape = C.shape[1:]
    if u_p is None:
        u_p = pad_velocity(u, prm.u_wall)
    C_p = pad_mirror_z(C)
    Gm = np.empty((3, 3) + shape)
    for a in range(3):
        for b in range(3):
            Gm[a, b] = 0.5 * (_shift(u_p[b], _E[a], shape)
                              - _shift(u_p[b], _NEG[a], shape))
    fP = peterlin(C, prm.L2[p])
    Cn = np.empty_like(C)
    for k, (kk, ll) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        adv = np.zeros(shape)
        for a in range(3):
            ua = u[a]
            back = C[k] - _shift(C_p[k], _NEG[a], shape)
            fwd = _shift(C_p[k], _E[a], shape) - C[k]
            adv += np.maximum(ua, 0.0) * back + np.minimum(ua, 0.0) * fwd
        S = np.zeros(shape)
        for m in range(3):
            S += C[_SYM[(kk, m)]] * Gm[m, ll] + Gm[m, kk] * C[_SYM[(m, ll)]]
        delta = 1.0 if kk == ll else 0.0
        Cn[k] = C[k] + (-adv + S - (fP * C[k] - delta) / prm.tau_P[p])
    return Cn


def stream(fstar, rho, prm: Params):
    """Periodic streaming in x and y; links that leave through z = -1/2 or
    z = nz - 1/2 are bounced back at the same node with the moving-wall
    correction -6 w_i rho_s(x) c_i.u_wall (rho_s of the pre-collision state
    of this step)."""
    nz, ny, nx = fstar.shape[2:]
    out = np.empty_like(fstar)
    ix = np.arange(nx)
    iy = np.arange(ny)
    for i in range(Q):
        cx, cy, cz = (int(v) for v in CV[i])
        src_x = (ix - cx) % nx
        src_y = (iy - cy) % ny
        moved = fstar[:, i][:, :, src_y][:, :, :, src_x]
        if cz == 0:
            out[:, i] = moved
            continue
        if cz > 0:
            out[:, i, 1:] = moved[:, :-1]
            z = 0                       # source plane z - 1 is the bottom wall
        else:
            out[:, i, :-1] = moved[:, 1:]
            z = nz - 1                  # source plane z + 1 is the top wall
        # the population arriving in direction i is the one that left this
        # node in direction opp(i) and was reflected by the wall
        o = OPP[i]
        uw = prm.u_wall if CV[o, 2] > 0 else -prm.u_wall
        cu = CV[o, 0] * uw
        out[:, i, z] = fstar[:, o, z] - 6.0 * W[o] * rho[:, z] * cu
    return out


# --------------------------------------------------------------------------
class Oracle:
    """FP64 reference solver.  State: post-stream populations f[2][19][z][y][x]
    and the conformation tensor C[6][z][y][x] (xx, yy, zz, xy, xz, yz)."""

    def __init__(self, params: dict, f=None, C=None):
        self.prm = Params(params)
        p = self.prm
        shape = (p.nz, p.ny, p.nx)
        self.shape = shape
        self.step_count = 0
        self.status = 0
        if f is None:
            z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny),
                                  np.arange(p.nx), indexing="ij")
            cx, cy, cz = p.centre
            inside = ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
                      < p.radius ** 2)
            rhoA = np.where(inside, p.rho_major, p.rho_minor)
            rhoB = np.where(inside, p.rho_minor, p.rho_major)
            if p.init_noise > 0.0:
                fac = init_noise_factors(p)
                rhoA, rhoB = rhoA * fac[0], rhoB * fac[1]
            f = np.empty((2, Q) + shape)
            for i in range(Q):
                f[0, i] = W[i] * rhoA
                f[1, i] = W[i] * rhoB
        self.f = np.array(f, dtype=np.float64, copy=True)
        if C is None:
            C = np.zeros((6,) + shape)
            C[0] = C[1] = C[2] = 1.0
        self.C = np.array(C, dtype=np.float64, copy=True)

    # ------------------------------------------------------------------
    def flow(self):
        """Moments, forces and velocities of the current state."""
        rho, j = moments(self.f)
        FA, FB = forces(rho, self.C, self.prm)
        ueqA, ueqB, u = velocities(rho, j, FA, FB, self.prm)
        return rho, j, FA, FB, ueqA, ueqB, u

    def step(self, n: int = 1):
        p = self.prm
        for _ in range(n):
            rho, _j, _FA, _FB, ueqA, ueqB, u = self.flow()
            if p.phase is not None:
                tr = self.C[0] + self.C[1] + self.C[2]
                if np.any(tr >= p.L2[p.phase]):
                    self.status |= STATUS_FENE
            fstar = collide(self.f, rho, ueqA, ueqB, p)
            if p.phase is not None:
                self.C = fene_p_update(self.C, u, p)
            self.f = stream(fstar, rho, p)
            if not (np.all(np.isfinite(self.f)) and np.all(np.isfinite(self.C))):
                self.status |= STATUS_NAN
            self.step_count += 1
        return self

    # ------------------------------------------------------------------
    def density(self):
        return self.f.sum(axis=1)

    def velocity(self):
        return self.flow()[6]
