"""Pins of the oracle's 1D barycentric interpolation (Section 3).

Independent of the oracle's own formulas: exact algebraic node values,
polynomial reproduction checked against numpy's power-basis evaluation, the
O(n^2) weight definition of eq. Barycentric-1D, and the Kronecker property.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_cheb():
    rows = []
    with open(os.path.join(GOLDEN, "chebyshev_points.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            n, k, s, w = line.split()
            val = eval(s, {"sqrt": math.sqrt})   # fixture expressions only
            rows.append((int(n), int(k), float(val), float(w)))
    return rows


def test_points_and_weights_match_closed_forms(orc):
    for n, k, s, w in _read_cheb():
        t = orc.cheb_points(n)
        assert abs(t[k] - s) <= 2 ** -52, (n, k, t[k], s)
        assert orc.bary_weights(n)[k] == w


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 9, 12])
def test_points_exactly_symmetric_and_descending(orc, n):
    t = orc.cheb_points(n)
    assert t[0] == 1.0 and t[n] == -1.0
    assert np.all(np.diff(t) < 0)
    assert np.array_equal(t, -t[::-1])
    if n % 2 == 0:
        assert t[n // 2] == 0.0
    assert np.max(np.abs(t - np.cos(np.arange(n + 1) * np.pi / n))) < 4e-16


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10])
def test_simple_weights_are_scaled_true_weights(orc, n):
    """w_k simple / w_k from the product definition is one common constant
    (the scale invariance of eq. Barycentric-1D)."""
    s = orc.cheb_points(n)
    true = np.array([1.0 / np.prod([s[k] - s[j] for j in range(n + 1) if j != k])
                     for k in range(n + 1)])
    ratio = orc.bary_weights(n) / true
    assert np.allclose(ratio, ratio[0], rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [1, 3, 6, 8, 10, 12])
@pytest.mark.parametrize("scale", [1.0, 1e-9, 1e-150, 1e150])
def test_polynomial_reproduction(orc, n, scale):
    """P1: sum_k p(s_k) L_k(t) = p(t) for deg p <= n on a mapped interval."""
    rng = np.random.default_rng(100 + n)
    a = scale * rng.uniform(-3, 3)
    b = a + scale * rng.uniform(0.5, 4)
    c, h = 0.5 * (a + b), 0.5 * (b - a)
    s = c + h * orc.cheb_points(n)
    coef = rng.uniform(-1, 1, n + 1)

    def p(t):   # polynomial in the local variable (t - c)/h
        return np.polynomial.polynomial.polyval((t - c) / h, coef)

    fk = p(s)
    for t in np.concatenate([rng.uniform(a, b, 40), [a, b, c]]):
        L = orc.lagrange_bary(n, s, t)
        got = float(np.dot(L, fk))
        ref = float(p(t))
        assert abs(got - ref) <= 1e-13 * np.sum(np.abs(coef)) * 10, (t, got, ref)


@pytest.mark.parametrize("n", [1, 4, 9])
def test_kronecker_at_nodes(orc, n):
    """L_k(s_j) = delta_jk exactly through the exact-hit rule (Algorithm 1)."""
    s = 0.3 + 1.7 * orc.cheb_points(n)
    for j in range(n + 1):
        L = orc.lagrange_bary(n, s, s[j])
        e = np.zeros(n + 1)
        e[j] = 1.0
        assert np.array_equal(L, e)


@pytest.mark.parametrize("n", [2, 5, 8])
def test_barycentric_equals_product_form(orc, n):
    rng = np.random.default_rng(n)
    s = -2.0 + 0.5 * orc.cheb_points(n)
    for t in rng.uniform(-2.5, -1.5, 30):
        Lb = orc.lagrange_bary(n, s, t)
        Lp = orc.lagrange_product(n, s, t)
        assert np.max(np.abs(Lb - Lp)) < 1e-13
        assert abs(np.sum(Lb) - 1.0) < 1e-14
