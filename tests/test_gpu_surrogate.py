"""Surrogate-network kernels (through the C ABI) against the FP64 reference on
the same bfloat16-rounded parameters: forward outputs, loss and gradient;
training reduces the loss; repeated training is bit-identical."""
import numpy as np
import pytest

import workloads as WL
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2181_amd import lbmve
    lbmve.lib()
    return torch, lbmve


def _init(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(mlp.SIZES[:-1], mlp.SIZES[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(rng.uniform(-0.1, 0.1, size=b))
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("n", [1, 17, 300])
def test_forward_loss_gradient_match_reference(env, n):
    torch, lbmve = env
    net = lbmve.Network(512)
    net.set_params(_init(1))
    pw = net.params(working=True)
    assert np.array_equal(pw, mlp.bf16_round(net.params()))
    x, t, m = WL.mlp_dataset(n, seed=n)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    md = torch.from_numpy(m).cuda()
    z = net.forward(xd).cpu().numpy()
    _, _, zr = mlp.forward(pw.astype(np.float64), x)
    assert np.abs(z - zr).max() <= 1e-5 * max(1.0, np.abs(zr).max())
    g, loss = net.gradient(xd, td, md)
    gr = mlp.gradient(pw.astype(np.float64), x, t, m)
    lr_ = mlp.loss(pw.astype(np.float64), x, t, m)
    assert abs(loss - lr_) <= 1e-5 * max(1.0, abs(lr_))
    err = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    assert err <= 1e-4, err
    net.close()


def test_training_reduces_loss_and_is_deterministic(env):
    torch, lbmve = env
    rng = np.random.default_rng(0)
    x = rng.normal(size=(400, 6)).astype(np.float32)
    t = np.stack([np.tanh(x[:, 0] - 0.5 * x[:, 1]), 0.3 * x[:, 2] * x[:, 3],
                  (x[:, 0] + x[:, 4] > 0).astype(np.float64)], axis=1).astype(np.float32)
    m = np.ones(400, dtype=np.float32)
    xd, td, md = (torch.from_numpy(a).cuda() for a in (x, t, m))
    finals = []
    for _ in range(2):
        net = lbmve.Network(400)
        net.set_params(_init(7))
        losses = [net.train_step(xd, td, md, 3e-3) for _ in range(300)]
        assert losses[-1] < 0.35 * losses[0], (losses[0], losses[-1])
        finals.append(net.params())
        net.close()
    assert np.array_equal(finals[0], finals[1])


def test_adam_step_matches_reference(env):
    torch, lbmve = env
    net = lbmve.Network(64)
    p0 = _init(3)
    net.set_params(p0)
    x, t, m = WL.mlp_dataset(64, seed=9)
    xd, td, md = (torch.from_numpy(a).cuda() for a in (x, t, m))
    g, _ = net.gradient(xd, td, md)
    net.train_step(xd, td, md, 1e-3)
    p1 = net.params()
    want, _, _ = mlp.adam(p0.astype(np.float64), g.astype(np.float64), np.zeros(p0.size),
                          np.zeros(p0.size), 1, lr=1e-3)
    assert np.abs(p1 - want).max() <= 1e-6
    net.close()
