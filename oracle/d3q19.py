"""D3Q19 lattice for the oracle (TEST INFRASTRUCTURE).

The paper models both fluids with a lattice-Boltzmann scheme (Section 2)
without naming the lattice; the reading used here is the 19-velocity cubic
lattice with sound speed c_s^2 = 1/3 and BGK relaxation.

Direction order (opposite pairs are (2k-1, 2k)):
    0 rest; 1,2 = +-x; 3,4 = +-y; 5,6 = +-z; 7,8 = +-(1,1,0);
    9,10 = +-(1,-1,0); 11,12 = +-(1,0,1); 13,14 = +-(1,0,-1);
    15,16 = +-(0,1,1); 17,18 = +-(0,1,-1)
Weights 1/3 (rest), 1/18 (|c| = 1), 1/36 (|c| = sqrt 2).
"""
import numpy as np

Q = 19

_HALF = [
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1),
]

C = np.zeros((Q, 3), dtype=np.int64)
for _k, _c in enumerate(_HALF):
    C[2 * _k + 1] = _c
    C[2 * _k + 2] = [-v for v in _c]

W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)

OPP = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, Q)])

CS2 = 1.0 / 3.0


def equilibrium(rho, u):
    """Second-order BGK equilibrium f^eq_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2
    - 3/2 u.u] for every direction; rho (..), u (3, ..) -> (Q, ..)."""
    rho = np.asarray(rho, dtype=np.float64)
    usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    out = np.empty((Q,) + rho.shape)
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
    return out
