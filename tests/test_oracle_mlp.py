"""Pins of the FP64 selector-network reference (oracle/mlp.py): gradients
against central finite differences of the loss, the closed form of the first
Adam step, and the layer algebra against an explicit per-row loop."""
import numpy as np
import pytest

from oracle import mlp


@pytest.mark.parametrize("k", [1, 7, 66])
def test_gradient_matches_finite_differences(k):
    rng = np.random.default_rng(k)
    p = mlp.init(k, seed=k) + rng.normal(scale=0.05, size=mlp.n_params(k))
    x = rng.normal(size=(9, mlp.NIN))
    t = rng.normal(size=(9, k))
    y, cache = mlp.forward(p, x, k)
    g = mlp.backward(p, x, cache, mlp.loss_grad(y, t), k)
    h = 1e-6
    idx = rng.choice(p.size, size=min(p.size, 300), replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp = mlp.loss(mlp.forward(p + e, x, k)[0], t)
        lm = mlp.loss(mlp.forward(p - e, x, k)[0], t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_forward_matches_row_loop():
    k = 5
    rng = np.random.default_rng(3)
    p = mlp.init(k, seed=3) + rng.normal(scale=0.1, size=mlp.n_params(k))
    x = rng.normal(size=(4, mlp.NIN))
    y, _ = mlp.forward(p, x, k)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, k)
    for r in range(4):
        h1 = [np.tanh(sum(W1[j, i] * x[r, i] for i in range(mlp.NIN)) + b1[j]) for j in range(mlp.NH)]
        h2 = [np.tanh(sum(W2[j, i] * h1[i] for i in range(mlp.NH)) + b2[j]) for j in range(mlp.NH)]
        for o in range(k):
            ref = sum(W3[o, i] * h2[i] for i in range(mlp.NH)) + b3[o]
            assert abs(y[r, o] - ref) < 1e-12


def test_first_adam_step_closed_form():
    """With m = v = 0, step 1 gives m_hat = g and v_hat = g^2, so the update
    is lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam(p, np.zeros(50), np.zeros(50), g, 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    k = 4
    rng = np.random.default_rng(5)
    x = rng.normal(size=(256, mlp.NIN))
    t = np.stack([np.sin(x[:, 0]) + 0.5 * x[:, 1] * (j + 1) for j in range(k)], axis=1)
    p = mlp.init(k, seed=2)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(mlp.forward(p, x, k)[0], t)
    for s in range(1, 301):
        y, c = mlp.forward(p, x, k)
        p, m, v = mlp.adam(p, m, v, mlp.backward(p, x, c, mlp.loss_grad(y, t), k), s, lr=3e-3)
    assert mlp.loss(mlp.forward(p, x, k)[0], t) < 0.05 * l0
