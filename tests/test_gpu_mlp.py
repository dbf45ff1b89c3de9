"""GPU selector-network kernels against the FP64 reference (oracle/mlp.py)
through the C ABI: forward values, loss gradient, parameter gradients (to
1e-4 relative per tensor, the FP32 rounding bar) and Adam steps."""
import numpy as np
import pytest

from oracle import mlp
from paper_1902_02250_amd import bltc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    bltc.load()
    return t


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("rows,k", [(1, 1), (33, 7), (1000, 66), (4096, 128)])
def test_forward_backward_vs_oracle(torch, rows, k):
    rng = np.random.default_rng(rows + k)
    p = mlp.init(k, seed=k) + rng.normal(scale=0.05, size=mlp.n_params(k))
    p = p.astype(np.float32).astype(np.float64)   # same parameters on both sides
    x = rng.normal(size=(rows, mlp.NIN)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(rows, k)).astype(np.float32).astype(np.float64)
    assert bltc.mlp_params(k) == mlp.n_params(k)
    y_ref, cache = mlp.forward(p, x, k)
    dy_ref = mlp.loss_grad(y_ref, t)
    g_ref = mlp.backward(p, x, cache, dy_ref, k)
    P, X, T = _t(torch, p), _t(torch, x), _t(torch, t)
    Y, C = bltc.mlp_forward(P, X, k)
    work = bltc.mlp_work(rows, k)
    dY, loss = bltc.mlp_loss(Y, T, work)
    G = bltc.mlp_backward(P, X, C, dY, work)
    torch.cuda.synchronize()
    assert _rel(Y.cpu().numpy(), y_ref) < 1e-5
    assert abs(loss.item() - mlp.loss(y_ref, t)) <= 1e-5 * mlp.loss(y_ref, t)
    assert _rel(dY.cpu().numpy(), dy_ref) < 1e-5
    g = G.cpu().numpy()
    o = 0
    for size in (64 * 12, 64, 64 * 64, 64, k * 64, k):
        assert _rel(g[o:o + size], g_ref[o:o + size]) < 1e-4, (o, size)
        o += size


def test_adam_vs_oracle(torch):
    rng = np.random.default_rng(9)
    n = 5000
    p = rng.normal(size=n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    P, M, V = _t(torch, p), _t(torch, m), _t(torch, v)
    # the kernel takes its constants in FP32: give the reference the same values
    b1, b2, lr, eps = (float(np.float32(c)) for c in (0.9, 0.999, 1e-2, 1e-8))
    for step in range(1, 6):
        g = rng.normal(size=n).astype(np.float32).astype(np.float64)
        p, m, v = mlp.adam(p, m, v, g, step, lr=lr, b1=b1, b2=b2, eps=eps)
        bltc.adam_step(P, M, V, _t(torch, g), step, lr, b1, b2, eps)
    torch.cuda.synchronize()
    assert _rel(P.cpu().numpy(), p) < 1e-6
    assert _rel(M.cpu().numpy(), m) < 1e-6 and _rel(V.cpu().numpy(), v) < 1e-5


def test_training_on_device_reduces_loss(torch):
    k = 8
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2048, mlp.NIN))
    t = np.stack([np.sin(x[:, 0]) + 0.3 * (j + 1) * x[:, 1] * x[:, 2] for j in range(k)], axis=1)
    P = _t(torch, mlp.init(k, seed=1))
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    X, T = _t(torch, x), _t(torch, t)
    work = bltc.mlp_work(2048, k)
    losses = []
    for step in range(1, 401):
        Y, C = bltc.mlp_forward(P, X, k)
        dY, loss = bltc.mlp_loss(Y, T, work)
        bltc.adam_step(P, M, V, bltc.mlp_backward(P, X, C, dY, work), step, 3e-3)
        if step in (1, 400):
            losses.append(loss.item())
    assert losses[1] < 0.1 * losses[0]
