"""Droplet observables for the oracle (TEST INFRASTRUCTURE).

The paper characterises the droplet by its deformation and orientation
(Introduction; Taylor's measure) and, for strongly deformed shapes, by the
projection L_p of the droplet length on the flow direction (Section 3, the
paragraph on elongation).  Readings:
  * phase field phi = (rho_A - rho_B)/(rho_A + rho_B), droplet weight
    w = max(phi, 0);
  * centroid X = sum w x / sum w and the 2x2 shear-plane inertia block
    I_ab = sum w (x_a - X_a)(x_b - X_b), a, b in {x, z};
  * D = (sqrt(l+) - sqrt(l-))/(sqrt(l+) + sqrt(l-)) from its eigenvalues,
    orientation theta = atan2(2 I_xz, I_xx - I_zz)/2 in degrees;
  * L_p = x_max - x_min + 1 over the nodes with phi > 0 (unwrapped x).
"""
from __future__ import annotations

import math

import numpy as np


def observe(f, C, u=None):
    """Observables of a state.  f (2, 19, nz, ny, nx); C (6, nz, ny, nx);
    u (3, nz, ny, nx) the physical velocity if max|u| is wanted."""
    rho = f.sum(axis=1)
    rhoA, rhoB = rho[0], rho[1]
    nz, ny, nx = rhoA.shape
    phi = (rhoA - rhoB) / (rhoA + rhoB)
    w = np.maximum(phi, 0.0)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64),
                          np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    sw = w.sum()
    out = dict(mass=(float(rhoA.sum()), float(rhoB.sum())), weight=float(sw))
    if sw > 0.0:
        X = (w * x).sum() / sw
        Y = (w * y).sum() / sw
        Z = (w * z).sum() / sw
        dx, dz = x - X, z - Z
        Ixx = (w * dx * dx).sum()
        Ixz = (w * dx * dz).sum()
        Izz = (w * dz * dz).sum()
        mean = 0.5 * (Ixx + Izz)
        rad = math.sqrt((0.5 * (Ixx - Izz)) ** 2 + Ixz ** 2)
        lp, lm = mean + rad, max(mean - rad, 0.0)
        D = (math.sqrt(lp) - math.sqrt(lm)) / (math.sqrt(lp) + math.sqrt(lm))
        theta = 0.5 * math.degrees(math.atan2(2.0 * Ixz, Ixx - Izz))
        out.update(centroid=(float(X), float(Y), float(Z)), D=D, theta_deg=theta,
                   inertia=(float(Ixx), float(Ixz), float(Izz)))
    inside = np.any(phi > 0.0, axis=(0, 1))
    xs = np.nonzero(inside)[0]
    out["Lp"] = float(xs.max() - xs.min() + 1) if xs.size else 0.0
    out["trC_max"] = float((C[0] + C[1] + C[2]).max())
    if u is not None:
        out["umax"] = float(np.sqrt((u * u).sum(axis=0)).max())
    return out
