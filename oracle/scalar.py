"""Node-by-node pure-Python oracle for tiny lattices (TEST INFRASTRUCTURE).

An independent, deliberately literal second implementation of the same
discrete step as oracle.solver (the readings are listed there).  It builds
the 19-velocity lattice by enumerating the cube {-1,0,1}^3 (|c|^2 <= 2, weight
by speed), loops over nodes and directions explicitly and applies the ghost
rules through explicit index functions.  It exists only to check the
array-at-a-time oracle on lattices of a few dozen nodes.
"""
from __future__ import annotations


def _lattice():
    # enumerate the D3Q19 velocities and put them in the documented order
    vel = []
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                if cx * cx + cy * cy + cz * cz <= 2:
                    vel.append((cx, cy, cz))
    order = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
             (0, 0, 1), (0, 0, -1), (1, 1, 0), (-1, -1, 0), (1, -1, 0),
             (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
             (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    assert sorted(order) == sorted(vel)
    weight = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    w = [weight[cx * cx + cy * cy + cz * cz] for (cx, cy, cz) in order]
    opp = [order.index((-cx, -cy, -cz)) for (cx, cy, cz) in order]
    return order, w, opp


VEL, WT, OPPOSITE = _lattice()


def _feq(i, rho, u):
    cx, cy, cz = VEL[i]
    cu = cx * u[0] + cy * u[1] + cz * u[2]
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    return WT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _cidx(a, b):
    if a == b:
        return a
    lo, hi = min(a, b), max(a, b)
    return {(0, 1): 3, (0, 2): 4, (1, 2): 5}[(lo, hi)]


def scalar_step(f, Cf, prm):
    """One step on nested lists/arrays: f[s][i][z][y][x], Cf[k][z][y][x].
    ``prm`` is an oracle.solver.Params (plain numbers only are read).
    Returns new (f, C) as nested Python lists."""
    nx, ny, nz = prm.nx, prm.ny, prm.nz
    tau = prm.tau
    tau_m = prm.tau_minus   # odd-moment times (equal to tau under BGK)
    G = prm.G
    ph = prm.phase

    def wrap(x, y):
        return x % nx, y % ny

    rho = [[[[0.0] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(2)]
    jm = [[[[[0.0] * 3 for _ in range(nx)] for _ in range(ny)] for _ in range(nz)]
          for _ in range(2)]
    for s in range(2):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    r = 0.0
                    jj = [0.0, 0.0, 0.0]
                    for i in range(19):
                        v = float(f[s][i][z][y][x])
                        r += v
                        for a in range(3):
                            jj[a] += VEL[i][a] * v
                    rho[s][z][y][x] = r
                    jm[s][z][y][x] = jj

    def rho_at(s, x, y, z):
        # mirror ghost in z: the ghost plane repeats the boundary plane
        z = min(max(z, 0), nz - 1)
        x, y = wrap(x, y)
        return rho[s][z][y][x]

    def C_at(k, x, y, z):
        z = min(max(z, 0), nz - 1)
        x, y = wrap(x, y)
        return float(Cf[k][z][y][x])

    def stress_at(k, x, y, z):
        rA, rB = rho_at(0, x, y, z), rho_at(1, x, y, z)
        frac = (rA if ph == 0 else rB) / (rA + rB)
        chi = (frac - prm.chi_lo) / (prm.chi_hi - prm.chi_lo)
        chi = 0.0 if chi < 0.0 else (1.0 if chi > 1.0 else chi)
        tr = C_at(0, x, y, z) + C_at(1, x, y, z) + C_at(2, x, y, z)
        fp = (prm.L2[ph] - 3.0) / (prm.L2[ph] - tr)
        d = 1.0 if k < 3 else 0.0
        return chi * prm.eta_P[ph] / prm.tau_P[ph] * (fp * C_at(k, x, y, z) - d)

    def force_at(x, y, z):
        FA = [0.0, 0.0, 0.0]
        FB = [0.0, 0.0, 0.0]
        for i in range(1, 19):
            c = VEL[i]
            w3 = 3.0 * WT[i]
            nB = rho_at(1, x + c[0], y + c[1], z + c[2])
            nA = rho_at(0, x + c[0], y + c[1], z + c[2])
            for a in range(3):
                FA[a] += w3 * nB * c[a]
                FB[a] += w3 * nA * c[a]
        rA, rB = rho_at(0, x, y, z), rho_at(1, x, y, z)
        FA = [-G * rA * v for v in FA]
        FB = [-G * rB * v for v in FB]
        if ph is not None:
            unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
            for a in range(3):
                fpa = 0.0
                for b in range(3):
                    e = unit[b]
                    k = _cidx(a, b)
                    fpa += 0.5 * (stress_at(k, x + e[0], y + e[1], z + e[2])
                                  - stress_at(k, x - e[0], y - e[1], z - e[2]))
                FA[a] += rA / (rA + rB) * fpa
                FB[a] += rB / (rA + rB) * fpa
        return FA, FB

    ueq = [[[[None] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(2)]
    uph = [[[None] * nx for _ in range(ny)] for _ in range(nz)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                FA, FB = force_at(x, y, z)
                rA, rB = rho[0][z][y][x], rho[1][z][y][x]
                jA, jB = jm[0][z][y][x], jm[1][z][y][x]
                for a in range(3):
                    FA[a] += rA * prm.body_accel[a]
                    FB[a] += rB * prm.body_accel[a]
                den = rA / tau_m[0] + rB / tau_m[1]
                up = [(jA[a] / tau_m[0] + jB[a] / tau_m[1]) / den for a in range(3)]
                ueq[0][z][y][x] = [up[a] + tau_m[0] * FA[a] / rA for a in range(3)]
                ueq[1][z][y][x] = [up[a] + tau_m[1] * FB[a] / rB for a in range(3)]
                uph[z][y][x] = [(jA[a] + jB[a] + 0.5 * (FA[a] + FB[a])) / (rA + rB)
                                for a in range(3)]

    def post(s, i, x, y, z):
        fv = float(f[s][i][z][y][x])
        r, u = rho[s][z][y][x], ueq[s][z][y][x]
        if tau_m[s] == tau[s]:
            return fv - (fv - _feq(i, r, u)) / tau[s]
        # two relaxation times: the parts even and odd under i -> opposite(i)
        o = OPPOSITE[i]
        fo = float(f[s][o][z][y][x])
        even = 0.5 * (fv + fo) - 0.5 * (_feq(i, r, u) + _feq(o, r, u))
        odd = 0.5 * (fv - fo) - 0.5 * (_feq(i, r, u) - _feq(o, r, u))
        return fv - even / tau[s] - odd / tau_m[s]

    fn = [[[[[0.0] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(19)]
          for _ in range(2)]
    for s in range(2):
        for i in range(19):
            cx, cy, cz = VEL[i]
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        zs = z - cz
                        if 0 <= zs < nz:
                            xs, ys = wrap(x - cx, y - cy)
                            fn[s][i][z][y][x] = post(s, i, xs, ys, zs)
                        else:
                            o = OPPOSITE[i]
                            co = VEL[o]
                            uw = prm.u_wall if co[2] > 0 else -prm.u_wall
                            fn[s][i][z][y][x] = (post(s, o, x, y, z)
                                                 - 6.0 * WT[o] * rho[s][z][y][x]
                                                 * co[0] * uw)

    Cn = [[[[float(Cf[k][z][y][x]) for x in range(nx)] for y in range(ny)]
           for z in range(nz)] for k in range(6)]
    if ph is not None:
        def u_at(b, x, y, z):
            x, y = wrap(x, y)
            if z < 0:
                wall = -prm.u_wall if b == 0 else 0.0
                return 2.0 * wall - uph[0][y][x][b]
            if z >= nz:
                wall = prm.u_wall if b == 0 else 0.0
                return 2.0 * wall - uph[nz - 1][y][x][b]
            return uph[z][y][x][b]

        unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    Gm = [[0.5 * (u_at(b, x + unit[a][0], y + unit[a][1], z + unit[a][2])
                                  - u_at(b, x - unit[a][0], y - unit[a][1], z - unit[a][2]))
                           for b in range(3)] for a in range(3)]
                    u = uph[z][y][x]
                    tr = C_at(0, x, y, z) + C_at(1, x, y, z) + C_at(2, x, y, z)
                    fp = (prm.L2[ph] - 3.0) / (prm.L2[ph] - tr)
                    for k, (kk, ll) in enumerate(_PAIRS):
                        here = C_at(k, x, y, z)
                        adv = 0.0
                        for a in range(3):
                            e = unit[a]
                            back = here - C_at(k, x - e[0], y - e[1], z - e[2])
                            fwd = C_at(k, x + e[0], y + e[1], z + e[2]) - here
                            adv += max(u[a], 0.0) * back + min(u[a], 0.0) * fwd
                        S = 0.0
                        for m in range(3):
                            S += (C_at(_cidx(kk, m), x, y, z) * Gm[m][ll]
                                  + Gm[m][kk] * C_at(_cidx(m, ll), x, y, z))
                        d = 1.0 if kk == ll else 0.0
                        Cn[k][z][y][x] = here + (-adv + S - (fp * here - d) / prm.tau_P[ph])
    return fn, Cn

