"""FP64 reference of the per-batch (n, theta) selector network.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).  Not from the paper: the
paper fixes (theta, n, N0) by hand and notes that the values are not claimed
optimal (Section 6) and that the lower envelope of cost vs error gives the
most efficient parameters (Section 8.1); the selector learns that envelope
per target batch.

Network, with x the 12 normalised features of a batch:
    h1 = tanh(W1 x + b1)      (64)
    h2 = tanh(W2 h1 + b2)     (64)
    y  = W3 h2 + b3           (K: predicted log10 error of each candidate)
Loss over R rows: L = sum_{r,k} (y_rk - t_rk)^2 / (R K).
Adam (Kingma and Ba, 2015) with bias correction:
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Flat parameter layout: W1 [64][12], b1 [64], W2 [64][64], b2 [64],
W3 [K][64], b3 [K] (row-major), as the HIP kernels use.
"""
import numpy as np

NIN, NH = 12, 64


def n_params(k):
    return NH * NIN + NH + NH * NH + NH + k * NH + k


def unpack(p, k):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in ((NH, NIN), (NH,), (NH, NH), (NH,), (k, NH), (k,)):
        size = int(np.prod(shape))
        out.append(p[o:o + size].reshape(shape))
        o += size
    assert o == p.size
    return out


def forward(p, x, k):
    """Returns y (R, K) and the cache (h1, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, k)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y, (h1, h2)


def loss(y, t):
    return float(np.sum((y - t) ** 2) / y.size)


def loss_grad(y, t):
    return 2.0 * (y - t) / y.size


def backward(p, x, cache, dy, k):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(p, k)
    h1, h2 = cache
    x = np.asarray(x, dtype=np.float64)
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (p, m, v).  step counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(k, seed):
    """Seeded Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((NH, NIN), (NH, NH), (k, NH)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
