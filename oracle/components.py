"""Connected components of the droplet phase (TEST INFRASTRUCTURE).

Break-up (Section 3: the droplet splits into daughter droplets, binary or
with multiple neckings) is read as the number of connected components of the
set {phi > 0}, with face (6-) connectivity, periodic in x and y and bounded by
the walls in z.  Components smaller than a given node count are ignored.

Plain breadth-first search over the node graph; meant for lattices up to a
few hundred thousand nodes.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def component_sizes(mask):
    """Sizes of the 6-connected components of a boolean (nz, ny, nx) mask,
    periodic in x and y, sorted in decreasing order."""
    mask = np.asarray(mask, dtype=bool)
    nz, ny, nx = mask.shape
    seen = np.zeros_like(mask)
    sizes = []
    for start in zip(*np.nonzero(mask)):
        if seen[start]:
            continue
        seen[start] = True
        q = deque([start])
        n = 0
        while q:
            z, y, x = q.popleft()
            n += 1
            nbrs = (((z, y, (x + 1) % nx)), (z, y, (x - 1) % nx),
                    (z, (y + 1) % ny, x), (z, (y - 1) % ny, x),
                    (z + 1, y, x), (z - 1, y, x))
            for nz_, ny_, nx_ in nbrs:
                if 0 <= nz_ < nz and mask[nz_, ny_, nx_] and not seen[nz_, ny_, nx_]:
                    seen[nz_, ny_, nx_] = True
                    q.append((nz_, ny_, nx_))
        sizes.append(n)
    return sorted(sizes, reverse=True)


def count_components(f, min_size=1):
    """Number of droplet components of at least ``min_size`` nodes."""
    rho = f.sum(axis=1)
    phi = (rho[0] - rho[1]) / (rho[0] + rho[1])
    return sum(1 for s in component_sizes(phi > 0.0) if s >= min_size)
