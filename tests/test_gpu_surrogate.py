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


def test_trained_network_saves_search_runs(env):
    """What the trained network gains: with a known break-up threshold
    standing in for the simulations, searches that start from the network's
    proposed brackets need fewer runs and rounds than plain bisection over
    the window, and locate the same Ca_cr within the tolerance."""
    from paper_1411_2181_amd import sweep
    from paper_1411_2181_amd.surrogate import Surrogate

    def ca_cr(De, lam, c):
        return 0.16 + 0.02 * De + 0.05 * (lam - 1.0) + 0.2 * (c - 0.5)

    def run(specs):
        return [(sp.Ca > ca_cr(sp.De, sp.lam, sp.c), 0) for sp in specs], 0.0

    # inputs as in the study window: lambda = 0.8 / (1 - f) with polymer
    rng = np.random.default_rng(11)
    n = 600
    De = rng.choice([0.0, 0.5, 1.0, 2.0], size=n)
    fr = np.where(De > 0, rng.choice([0.2, 0.4], size=n), 0.0)
    lam = 0.8 / (1.0 - fr)
    c = rng.uniform(0.45, 0.65, size=n)
    Ca = rng.uniform(0.10, 0.26, size=n)
    L2 = rng.choice([100.0, 400.0], size=n)
    X = np.stack([Ca, De, lam, c, L2, fr], axis=1)
    cr = ca_cr(De, lam, c)
    broken = (Ca > cr).astype(float)
    D = 0.6 * Ca / cr
    theta = 45.0 - 80.0 * Ca
    sg = Surrogate(batch_max=n, seed=1)
    losses = sg.fit(X, D, theta, broken, epochs=3000, lr=2e-3)
    assert losses[-1] < 0.2 * losses[0]

    tol, lo, hi = 0.02, 0.10, 0.26
    qs = WL.query_window(16)
    for q in qs:
        q["lam"] = 0.8 / (1.0 - q["polymer_fraction"])
    plain = [sweep.Search(q["De"], q["lam"], q["confinement"], 24.0, lo, hi, hard_lo=lo, hard_hi=hi)
             for q in qs]
    prop = []
    for q in qs:
        b = sg.propose(q["De"], q["lam"], q["confinement"], lo, hi, tol=tol)
        blo, bhi = b if b is not None else (lo, hi)
        prop.append(sweep.Search(q["De"], q["lam"], q["confinement"], 24.0, blo, bhi,
                                 hard_lo=lo, hard_hi=hi, speculate=b is not None))
    sg.close()
    plain, _, r_plain = sweep.bisect(plain, tol=tol, run=run)
    prop, _, r_prop = sweep.bisect(prop, tol=tol, run=run)
    runs_plain = sum(s.runs for s in plain)
    runs_prop = sum(s.runs for s in prop)
    print(f"plain: {runs_plain} runs, {r_plain} rounds; surrogate: {runs_prop} runs, {r_prop} rounds")
    for a, b, q in zip(plain, prop, qs):
        t = ca_cr(q["De"], q["lam"], q["confinement"])
        assert a.outside == b.outside
        if t < hi:
            assert a.lo <= t < a.hi and b.lo <= t < b.hi
            assert abs(a.ca_cr - b.ca_cr) <= tol * 1.000001
    assert runs_prop <= 0.8 * runs_plain
    assert r_prop < r_plain
