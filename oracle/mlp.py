"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE).

The surrogate maps six run parameters (Ca, De, lambda, 2R/W, L^2, polymer
fraction; the dimensionless groups of Section 2 and the set-up of Section 3)
to (steady deformation D, orientation, break-up logit).  Network: 6 -> 128
-> 128 -> 3, tanh hidden units, linear outputs.  Loss per batch of n rows:

    L = (1/n) sum_r [ m_r (e0^2 + e1^2)/2 + softplus(z2) - t2 z2 ],
    e_k = z_k - t_k,

m_r = 1 for runs that did not break (D and angle are defined only then),
t2 in {0, 1} the break-up label.  Forward and backward here use exactly the
weights they are given (the GPU path passes its bf16-rounded copies) and
accumulate in float64.

Parameter vector (float32 master order): W1[6][128], b1[128], W2[128][128],
b2[128], W3[128][3], b3[3]; W[k][j] multiplies input k into unit j.
"""
from __future__ import annotations

import numpy as np

SIZES = (6, 128, 128, 3)


def n_params(sizes=SIZES):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(p, sizes=SIZES):
    out, k = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = np.asarray(p[k:k + a * b], dtype=np.float64).reshape(a, b)
        k += a * b
        bias = np.asarray(p[k:k + b], dtype=np.float64)
        k += b
        out.append((W, bias))
    return out


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float32)


def forward(p, x):
    """Activations of every layer: x (n, 6) -> (h1, h2, z)."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    z = h2 @ W3 + b3
    return h1, h2, z


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def loss(p, x, t, m):
    _, _, z = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    e = z[:, :2] - t[:, :2]
    per = 0.5 * m * (e[:, 0] ** 2 + e[:, 1] ** 2) + softplus(z[:, 2]) - t[:, 2] * z[:, 2]
    return float(per.mean())


def gradient(p, x, t, m):
    """dL/dp by backpropagation, same layout as p."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    n = x.shape[0]
    h1, h2, z = forward(p, x)
    d = np.empty_like(z)
    d[:, 0] = m * (z[:, 0] - t[:, 0])
    d[:, 1] = m * (z[:, 1] - t[:, 1])
    d[:, 2] = 1.0 / (1.0 + np.exp(-z[:, 2])) - t[:, 2]
    d /= n
    gW3 = h2.T @ d
    gb3 = d.sum(axis=0)
    dz2 = (d @ W3.T) * (1.0 - h2 * h2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 * h1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam(p, g, mom, vel, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, mom, vel)."""
    mom = b1 * mom + (1.0 - b1) * g
    vel = b2 * vel + (1.0 - b2) * g * g
    mh = mom / (1.0 - b1 ** step)
    vh = vel / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), mom, vel
