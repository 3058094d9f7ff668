"""Learned surrogate that proposes Ca_cr brackets (host driver).

The network (include/lbmve_surrogate.h; kernels in csrc/sg_kernels.hip)
maps the six run parameters (Ca, De, lambda, 2R/W, L^2, polymer fraction)
to (steady D, orientation / 45 degrees, break-up logit).  It is trained on
runs the solver itself produced, and only *proposes* where to bracket the
critical capillary number: both ends of a proposed bracket are verified by
full simulations (sweep.bisect), and a bracket end that fails moves the
search outward until simulations confirm a bracket.
"""
from __future__ import annotations

import numpy as np

from . import lbmve

N_IN = 6


def glorot(seed: int, sizes=(6, 128, 128, 3)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


class Surrogate:
    def __init__(self, batch_max: int = 4096, seed: int = 0, device="cuda:0"):
        self.net = lbmve.Network(batch_max, device=device)
        self.net.set_params(glorot(seed))
        self.mu = np.zeros(N_IN, np.float32)
        self.sd = np.ones(N_IN, np.float32)
        self.device = device

    def _x(self, inputs):
        import torch
        x = (np.asarray(inputs, np.float32) - self.mu) / self.sd
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(self.device)

    def fit(self, inputs, D, theta_deg, broken, epochs: int = 2000, lr: float = 3e-3,
            batch: int | None = None, seed: int = 0):
        """Full-batch (or minibatch) Adam on the masked-MSE + BCE loss.
        Targets: D, theta/45, broken in {0, 1}; D and theta only count for
        runs that did not break."""
        import torch
        X = np.asarray(inputs, np.float32)
        self.mu = X.mean(axis=0)
        self.sd = X.std(axis=0) + 1e-6
        br = np.asarray(broken, np.float32)
        Dv = np.nan_to_num(np.asarray(D, np.float32))
        Tv = np.nan_to_num(np.asarray(theta_deg, np.float32)) / 45.0
        T = np.stack([Dv, Tv, br], axis=1).astype(np.float32)
        M = (1.0 - br).astype(np.float32)
        n = X.shape[0]
        bs = n if batch is None else min(batch, n)
        rng = np.random.default_rng(seed)
        xd = self._x(X)
        td = torch.from_numpy(T).to(self.device)
        md = torch.from_numpy(M).to(self.device)
        losses = []
        for _ in range(epochs):
            if bs == n:
                losses.append(self.net.train_step(xd, td, md, lr))
            else:
                idx = torch.from_numpy(rng.choice(n, size=bs, replace=False)).to(self.device)
                losses.append(self.net.train_step(xd[idx].contiguous(), td[idx].contiguous(),
                                                  md[idx].contiguous(), lr))
        return losses

    def predict(self, inputs):
        z = self.net.forward(self._x(inputs)).cpu().numpy().astype(np.float64)
        p = 1.0 / (1.0 + np.exp(-z[:, 2]))
        return z[:, 0], 45.0 * z[:, 1], p

    def breakup_probability(self, Ca, De, lam, c, L2=100.0, fraction=0.4):
        Ca = np.atleast_1d(np.asarray(Ca, dtype=np.float64))
        X = np.stack([Ca, np.full(Ca.size, De), np.full(Ca.size, lam), np.full(Ca.size, c),
                      np.full(Ca.size, L2), np.full(Ca.size, fraction)], axis=1)
        return self.predict(X)[2]

    def propose(self, De, lam, c, lo, hi, tol=0.02, L2=100.0, fraction=0.4, grid=512):
        """Bracket around the predicted break-up boundary on [lo, hi]: centred
        where the break-up probability crosses 1/2, half-width the larger of
        tol and half the distance between its 1/4 and 3/4 crossings (the
        network's own uncertainty), clipped to [lo, hi].  None when the
        network predicts no crossing in the range."""
        ca = np.linspace(lo, hi, grid)
        p = self.breakup_probability(ca, De, lam, c, L2, fraction)

        def crossing(level):
            above = np.nonzero(p >= level)[0]
            if above.size == 0:
                return None
            k = above[0]
            if k == 0:
                return float(ca[0])
            return float(ca[k - 1] + (ca[k] - ca[k - 1]) * (level - p[k - 1]) / max(p[k] - p[k - 1], 1e-12))

        mid = crossing(0.5)
        if mid is None:
            return None
        q1, q3 = crossing(0.25), crossing(0.75)
        q3 = hi if q3 is None else q3
        half = max(tol, 0.5 * (q3 - q1))
        return (max(lo, mid - half), min(hi, mid + half))

    def close(self):
        self.net.close()
