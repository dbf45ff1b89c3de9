"""Pins of the oracle's modified weights (eq. modified_weights, Algorithm 1).

Checks: the barycentric Algorithm 1 against the product-form Lagrange
polynomials (eq. Lagrange_polynomial) on tiny inputs; exactness on
polynomials of degree <= n in each variable (which contains partition of
unity and first moments); the exact-hit path; linearity.
"""
import numpy as np
import pytest

from paper_1902_02250_amd import inputs


@pytest.mark.parametrize("n", [1, 3, 6])
def test_alg1_equals_product_form(orc, n):
    pts = inputs.points("uniform", 64, 3)
    w = inputs.weights(64, 3)
    T = orc.Tree(pts, 10)
    a = T.modified_weights(w, n, form=0)
    b = T.modified_weights(w, n, form=1)
    # the product form needs distinct nodes: skip clusters with a flat side
    ok = np.all(T.box[:, 3:] > T.box[:, :3], axis=1)
    assert ok.sum() >= T.nnodes // 2
    assert np.max(np.abs(a[ok] - b[ok])) <= 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_polynomial_moments(orc, n):
    """sum_k p(s_k) fhat_k = sum_j p(y_j) f_j for p in Q_n, per cluster: the
    interpolant of p is p itself (uniqueness, Section 2)."""
    pts = inputs.points("mixture", 3000, 4)
    w = inputs.weights(3000, 4)
    T = orc.Tree(pts, 200)
    fh = T.modified_weights(w, n)
    g = T.grids(n)
    rng = np.random.default_rng(n)
    degs = rng.integers(0, n + 1, size=(6, 3))
    degs[0] = 0            # partition of unity
    degs[1] = [1, 0, 0]    # first moments
    degs[2] = [0, 0, 1]
    degs[3] = [n, n, n]
    for q in range(T.nnodes):
        idx = T.perm[T.pbegin[q]:T.pend[q]]
        c = T.center[q]
        for e in degs:
            pj = np.prod([(pts[a, idx] - c[a]) ** e[a] for a in range(3)], axis=0)
            lhs = np.einsum("i,j,k,cijk->c", (g[q, 0] - c[0]) ** e[0], (g[q, 1] - c[1]) ** e[1],
                            (g[q, 2] - c[2]) ** e[2], fh[q])
            rhs = w[:, idx] @ pj
            scale = np.abs(w[:, idx]) @ np.abs(pj) + 1e-300
            assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale), (q, e, lhs, rhs)


def test_particle_on_a_node(orc):
    """A particle sitting exactly on a mapped grid point puts its whole weight
    on that grid point (the exact-hit branch of Algorithm 1)."""
    n = 4
    lo, hi = np.array([-1.0, -0.5, 0.25]), np.array([1.0, 1.5, 2.25])
    t = orc.cheb_points(n)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    s = c[:, None] + h[:, None] * t[None, :]
    # two corner particles fix the tight box; the third sits on node (1, 2, 3)
    pts = np.array([lo, hi, [s[0, 1], s[1, 2], s[2, 3]]]).T
    w = np.array([[0.0, 0.0, 2.0], [0.0, 0.0, -1.0], [0.0, 0.0, 0.5]])
    T = orc.Tree(pts, 10)
    assert np.array_equal(T.box[0], np.concatenate([lo, hi]))
    fh = T.modified_weights(w, n)
    expect = np.zeros((3, n + 1, n + 1, n + 1))
    expect[:, 1, 2, 3] = [2.0, -1.0, 0.5]
    assert np.array_equal(fh[0], expect)
    # a particle on a face node in one axis only: delta in that axis
    pts2 = np.array([lo, hi, [0.1, s[1, 0], 0.7]]).T
    fh2 = T.__class__(pts2, 10).modified_weights(w, n)
    assert np.all(fh2[0][:, :, 1:, :] == 0.0)


def test_weights_linear(orc):
    pts = inputs.points("uniform", 2000, 9)
    f = inputs.weights(2000, 9)
    g = inputs.weights(2000, 10)
    T = orc.Tree(pts, 150)
    a = T.modified_weights(2.0 * f - 3.0 * g, 5)
    b = 2.0 * T.modified_weights(f, 5) - 3.0 * T.modified_weights(g, 5)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
