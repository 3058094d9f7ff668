"""Physical groups -> lattice parameters of one run (host logic).

The paper describes each run by the capillary number Ca = eta_M gamma_dot R/
sigma (Introduction), the Deborah number, the viscosity ratio lambda set on
total (solvent + polymer) viscosity with the polymer in one phase only and a
polymer fraction of about 0.4 (Section 2, the MV/DV paragraph), the
confinement 2R/W and the extensibility L^2; the shear rate is
gamma_dot = 2 U_w / W (nomenclature) and the emulsion time is
tau_em = R eta_M / sigma (Eq. (9)).

Lattice readings:
  * kinematic viscosity of a BGK component (tau - 1/2)/3; dynamic viscosity
    eta_s = rho_ref (tau_s - 1/2)/3 with rho_ref = rho_major + rho_minor;
  * droplet viscoelastic (DV): eta_d = eta_A + eta_P = lambda eta_B,
    eta_P = fraction * eta_d; matrix viscoelastic (MV): eta_M = eta_B + eta'_P,
    eta'_P = fraction * eta_M, eta_A = lambda eta_M;
  * Deborah number De = tau_P gamma_dot, so tau_P = De / gamma_dot; the
    paper's Oldroyd-B form De = (tau_P / tau_em)(eta_P / eta_M) (Eq. (8)) is
    reported beside it;
  * U_w = gamma_dot W / 2 with gamma_dot = Ca sigma / (eta_M R); sigma comes
    from the Laplace calibration of the same (G, densities, tau) set.
"""
from __future__ import annotations

import json
import math
import os

RHO_MAJOR = 1.0
RHO_MINOR = 0.04
# Shan-Chen coupling of the mapped workloads.  With the velocity-shift
# forcing the minority densities and the interface depend on tau; droplets
# stay Laplace-consistent only for tau of about 1..1.75, which caps the
# viscosity and hence the Ca reachable at a given wall speed.  G = 0.75 (a
# shallower quench than the 0.9 of the small parity case) lowers sigma by
# ~25 % and so raises the reachable Ca by as much.
G_DEFAULT = 0.75
TAU_MAX = 1.75
CS2 = 1.0 / 3.0

_HERE = os.path.dirname(os.path.abspath(__file__))
SIGMA_TABLE = os.path.join(_HERE, "sigma_table.json")


def eta_of_tau(tau: float, rho_ref: float = RHO_MAJOR + RHO_MINOR) -> float:
    return rho_ref * CS2 * (tau - 0.5)


def tau_of_eta(eta: float, rho_ref: float = RHO_MAJOR + RHO_MINOR) -> float:
    return eta / (rho_ref * CS2) + 0.5


def sigma_for(tau_A: float, tau_B: float, G: float = G_DEFAULT) -> float:
    """Surface tension at (G, tau_A, tau_B): bilinear interpolation in the
    calibrated (tau_A, tau_B) grid of the nearest G (the Shan-Chen interface
    depends on tau); raises outside the usable part of the grid."""
    with open(SIGMA_TABLE) as fh:
        table = json.load(fh)
    Gs = sorted({e["G"] for e in table["entries"]})
    g = min(Gs, key=lambda v: abs(v - G))
    if abs(g - G) > 1e-9:
        raise ValueError(f"no sigma calibration for G = {G}")
    grid = {(e["tau_A"], e["tau_B"]): e for e in table["entries"] if e["G"] == g}
    ta_s = sorted({k[0] for k in grid})
    tb_s = sorted({k[1] for k in grid})

    def bracket(v, axis):
        if v <= axis[0]:
            return axis[0], axis[0], 0.0
        if v >= axis[-1]:
            return axis[-1], axis[-1], 0.0
        for lo, hi in zip(axis[:-1], axis[1:]):
            if lo <= v <= hi:
                return lo, hi, (v - lo) / (hi - lo)
        raise ValueError(v)

    a0, a1, fa = bracket(tau_A, ta_s)
    b0, b1, fb = bracket(tau_B, tb_s)
    val = 0.0
    for (ta, wa) in ((a0, 1 - fa), (a1, fa)):
        for (tb, wb) in ((b0, 1 - fb), (b1, fb)):
            if wa * wb == 0.0:
                continue
            e = grid[(ta, tb)]
            if not e.get("usable", True):
                raise ValueError(f"tau pair ({ta}, {tb}) at G = {g} is outside the stable range")
            val += wa * wb * e["sigma"]
    return float(val)


def lattice_params(nx: int, ny: int, nz: int, R: float, Ca: float, De: float, lam: float,
                   phase: str = "DV", L2: float = 100.0, fraction: float = 0.4,
                   tau_matrix: float = 1.0, sigma: float | None = None,
                   G: float = G_DEFAULT, u_max: float = 0.1) -> dict:
    """Lattice parameter dictionary (names of lbm_params) for a run.

    ``tau_matrix`` sets the matrix solvent relaxation time; if the resulting
    wall speed exceeds ``u_max`` the viscosities are raised (tau_matrix
    increased) until it does not, keeping every dimensionless group fixed.
    """
    rho_ref = RHO_MAJOR + RHO_MINOR
    W = float(nz)
    tau_B = tau_matrix
    for _ in range(64):
        eta_B = eta_of_tau(tau_B, rho_ref)
        if phase == "DV":
            eta_M = eta_B
            eta_d = lam * eta_M
            eta_P = fraction * eta_d
            eta_A = eta_d - eta_P
            eta_Ps = (eta_P, 0.0)
        elif phase == "MV":
            eta_M = eta_B / (1.0 - fraction)
            eta_P = fraction * eta_M
            eta_A = lam * eta_M
            eta_Ps = (0.0, eta_P)
        elif phase == "N":
            eta_M = eta_B
            eta_A = lam * eta_M
            eta_Ps = (0.0, 0.0)
        else:
            raise ValueError(phase)
        tau_A = tau_of_eta(eta_A, rho_ref)
        sig = sigma if sigma is not None else sigma_for(tau_A, tau_B, G)
        gdot = Ca * sig / (eta_M * R)
        u_wall = gdot * W / 2.0
        if u_wall <= u_max and tau_A > 0.5 + 1e-3:
            break
        tau_B = 0.5 + (tau_B - 0.5) * min(1.25, max(1.05, u_wall / u_max))
        if tau_B > TAU_MAX:
            raise ValueError("no admissible lattice parameters (tau would exceed "
                             f"{TAU_MAX} for U_w <= {u_max})")
    else:
        raise ValueError("no admissible lattice parameters")
    if max(tau_A, tau_B) > TAU_MAX:
        raise ValueError(f"tau = ({tau_A:.3f}, {tau_B:.3f}) outside the stable range")
    if De > 0.0 and phase in ("DV", "MV"):
        tau_P = De / gdot
    else:
        tau_P = 1.0
        eta_Ps = (0.0, 0.0)
    p = dict(nx=int(nx), ny=int(ny), nz=int(nz), u_wall=u_wall, radius=float(R),
             cx=-1.0, cy=-1.0, cz=-1.0, rho_major=RHO_MAJOR, rho_minor=RHO_MINOR, G=G,
             tau=(tau_A, tau_B), tau_P=(tau_P, tau_P), eta_P=eta_Ps, L2=(L2, L2),
             chi_lo=0.0, chi_hi=0.0)
    tau_em = R * eta_M / sig
    info = dict(sigma=sig, gamma_dot=gdot, eta_M=eta_M, tau_em=tau_em,
                De_oldroyd=(tau_P / tau_em) * (fraction if phase == "MV" else
                                               fraction * lam) if De > 0 else 0.0,
                Re=RHO_MAJOR * gdot * R * R / eta_M)
    return p, info


def run_length(tau_em: float, lo: int = 10000, hi: int = 40000) -> int:
    """Steps to t / tau_em = 100 (the paper's last snapshot), clamped."""
    return int(min(hi, max(lo, round(100.0 * tau_em))))


def taylor_deformation(Ca: float, lam: float) -> float:
    """Taylor's small-deformation law D = Ca (19 lambda + 16)/(16 lambda + 16)."""
    return Ca * (19.0 * lam + 16.0) / (16.0 * lam + 16.0)
