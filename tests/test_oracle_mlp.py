"""Pins of the FP64 surrogate-network reference: backpropagation against
central finite differences, bfloat16 rounding against hand-worked values,
and one Adam step against its closed form."""
import numpy as np

import workloads as WL
from oracle import mlp


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=mlp.n_params()) * scale).astype(np.float64)


def test_param_count():
    assert mlp.n_params() == 6 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 == 17795


def test_backprop_matches_finite_differences():
    p = _params(1)
    x, t, m = WL.mlp_dataset(7, seed=3)
    g = mlp.gradient(p, x, t, m)
    rng = np.random.default_rng(5)
    idx = rng.choice(p.size, size=60, replace=False)
    # include a few of each block (W1, b1, W2, b2, W3, b3)
    idx = np.concatenate([idx, [0, 770, 900, 17000, 17400, 17794]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, x, t, m) - mlp.loss(pm, x, t, m)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_masked_rows_carry_no_regression_gradient():
    p = _params(2)
    x, t, m = WL.mlp_dataset(5, seed=4)
    m[:] = 0.0
    t2 = t.copy()
    t2[:, :2] += 10.0            # regression targets are ignored where masked
    assert np.allclose(mlp.gradient(p, x, t, m), mlp.gradient(p, x, t2, m), rtol=0, atol=0)


def test_bf16_rounding_hand_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8,
                     -2.5, 3.0e38, 0.0], dtype=np.float32)
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 2.9980e38, 0.0])
    got = mlp.bf16_round(vals).astype(np.float64)
    # exact for the first five; the large value rounds to the nearest bf16
    assert np.array_equal(got[:5], want[:5])
    assert abs(got[5] / 3.0e38 - 1) < 2 ** -8
    assert got[6] == 0.0


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    p1, m1, v1 = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # first bias-corrected step: m/sqrt(v) = sign(g) (up to eps)
    assert np.allclose(p1[:2], p[:2] - 0.01 * np.sign(g[:2]), rtol=0, atol=1e-9)
    assert p1[2] == p[2]
