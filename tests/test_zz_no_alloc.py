"""The allocation-free surrogate gradient (sg_gradient_noalloc, for callers
that cannot allocate device memory) against sg_gradient on the same network
and rows: two calls in a row, the second with fewer rows, both bit-identical
to the workspace path; rows beyond the fixed scratch are rejected."""
import numpy as np
import pytest

import workloads as WL
from oracle import mlp

pytestmark = pytest.mark.gpu


def _init(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(mlp.SIZES[:-1], mlp.SIZES[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(rng.uniform(-0.1, 0.1, size=b))
    return np.concatenate(parts).astype(np.float32)


def test_gradient_without_allocation_matches_workspace_path():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2181_amd import lbmve
    lbmve.lib()
    net = lbmve.Network(lbmve.SG_NOALLOC_MAX_ROWS + 8)
    net.set_params(_init(3))
    grad = torch.empty(net.n_params, dtype=torch.float32, device=net.device)
    loss = torch.empty(1, dtype=torch.float32, device=net.device)
    for n in (lbmve.SG_NOALLOC_MAX_ROWS, 37):       # the second call has fewer rows
        print(f"case noalloc gradient, {n} rows", flush=True)
        x, t, m = WL.mlp_dataset(n, seed=100 + n)
        xd, td, md = (torch.tensor(a, dtype=torch.float32, device=net.device) for a in (x, t, m))
        grad.fill_(np.nan)
        loss.fill_(np.nan)
        net.gradient_noalloc(xd, td, md, grad, loss)
        torch.cuda.synchronize()
        g_ref, l_ref = net.gradient(xd, td, md)
        g = grad.cpu().numpy()
        assert np.array_equal(g, g_ref), n
        assert float(loss.cpu()[0]) == l_ref
        assert np.abs(g).max() > 0.0
    # more rows than the fixed scratch holds: rejected on the host
    n = lbmve.SG_NOALLOC_MAX_ROWS + 1
    x, t, m = WL.mlp_dataset(n, seed=7)
    xd, td, md = (torch.tensor(a, dtype=torch.float32, device=net.device) for a in (x, t, m))
    with pytest.raises(lbmve.LbmError):
        net.gradient_noalloc(xd, td, md, grad, loss)
    net.close()
