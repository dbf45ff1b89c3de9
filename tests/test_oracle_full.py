"""Pins of the oracle's full regularized Stokeslet + rotlet kernel
(eq. MRS_2: forces and torques to linear and angular velocity) against the
separately pinned Stokeslet and rotlet: the four blocks of the 6 x 6 kernel,
linearity, and the treecode with six weight components."""
import numpy as np
import pytest

from paper_1902_02250_amd import inputs


def test_full_pair_blocks(orc):
    """(f, 0) gives the Stokeslet in u and, in w, the rotlet's velocity block
    with n -> f (both are 1/2 Q (. x d)); (0, n) gives the rotlet."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        x, y = rng.normal(size=3), rng.normal(size=3)
        f, n = rng.normal(size=3), rng.normal(size=3)
        eps = rng.uniform(0.01, 0.5)
        uf = orc.pair("full", x, y, np.concatenate([f, 0 * n]), eps)
        un = orc.pair("full", x, y, np.concatenate([0 * f, n]), eps)
        assert np.allclose(uf[:3], orc.pair("stokeslet", x, y, f, eps), rtol=1e-14, atol=0)
        assert np.allclose(uf[3:], orc.pair("rotlet", x, y, f, eps)[:3], rtol=1e-14, atol=0)
        assert np.allclose(un, orc.pair("rotlet", x, y, n, eps), rtol=1e-14, atol=0)
        both = orc.pair("full", x, y, np.concatenate([f, n]), eps)
        assert np.allclose(both, uf + un, rtol=1e-13, atol=1e-15)


def test_full_treecode_and_direct(orc):
    pts = inputs.points("mixture", 3000, 13)
    w = np.concatenate([inputs.weights(3000, 13), inputs.weights(3000, 14)])
    d = orc.direct("full", pts, pts, w, eps=0.05)
    ds = orc.direct("stokeslet", pts, pts, w[:3], eps=0.05)
    dr = orc.direct("rotlet", pts, pts, w[3:], eps=0.05)
    drf = orc.direct("rotlet", pts, pts, w[:3], eps=0.05)
    # same pairs, summed in another grouping: rounding only
    assert orc.rel_l2(d[:3], ds + dr[:3]) < 1e-13
    assert orc.rel_l2(d[3:], drf[:3] + dr[3:]) < 1e-13
    t, npx, ndr = orc.treecode("full", pts, pts, w, 0.05, 8, 0.6, 100, mac_mode=1,
                               order_leaf=32)
    assert npx > 0 and orc.rel_l2(d, t) < 1e-6
    t0, _, _ = orc.treecode("full", pts, pts, w, 0.05, 4, 0.0, 100, mac_mode=1, order_leaf=32)
    assert orc.rel_l2(d, t0) < 1e-13
