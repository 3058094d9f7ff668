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

    def propose(self, De, lam, c, lo, hi, L2=100.0, fraction=0.4, margin=0.02, grid=256):
        """Bracket [Ca_lo, Ca_hi] around the predicted break-up boundary
        (logit = 0) on [lo, hi], widened by ``margin`` on each side; None if
        the network predicts no crossing in the range."""
        ca = np.linspace(lo, hi, grid)
        X = np.stack([ca, np.full(grid, De), np.full(grid, lam), np.full(grid, c),
                      np.full(grid, L2), np.full(grid, fraction)], axis=1)
        _, _, p = self.predict(X)
        above = np.nonzero(p >= 0.5)[0]
        if above.size == 0:
            return None
        k = above[0]
        if k == 0:
            return (lo, min(hi, lo + 2 * margin))
        ca_star = ca[k - 1] + (ca[k] - ca[k - 1]) * (0.5 - p[k - 1]) / max(p[k] - p[k - 1], 1e-12)
        return (max(lo, ca_star - margin), min(hi, ca_star + margin))

    def close(self):
        self.net.close()
