"""Pins of the oracle's separation rule for the degree of each accepted
cluster (deg_min >= 1; an addition to the paper's fixed degree):
the Bernstein-ellipse criterion checked from the tree geometry in numpy,
minimality of the chosen degree, exactness for polynomial kernels of degree
at most deg_min (so every cluster reads the grid and weights of its own
degree), agreement with the fixed degree when the rule is off, and
convergence in the top degree."""
import numpy as np
import pytest

from paper_1902_02250_amd import inputs


def _kappa(rho):
    return rho / (1.0 + np.sqrt(1.0 - rho * rho))


@pytest.mark.parametrize("theta,degree,deg_min", [(0.7, 8, 1), (0.5, 6, 2), (0.9, 10, 3)])
def test_rule_degrees_follow_the_ellipse_criterion(orc, theta, degree, deg_min):
    src = inputs.points("mixture", 6000, 31)
    L = orc.lists(src, 150, src, theta, 64, 32, 512, degree=degree, deg_min=deg_min)
    T = orc.Tree(src, 150)
    _, bptr, bc, br = orc.batches(src, 64, 32, 512)
    pp, ids, deg = L["prox_ptr"], L["prox_ids"], L["prox_deg"]
    b = np.repeat(np.arange(pp.size - 1), np.diff(pp))
    rho = (br[b] + T.radius[ids]) / np.linalg.norm(bc[b] - T.center[ids], axis=1)
    lhs = np.log(np.maximum(_kappa(np.minimum(rho, 1.0)), 1e-300))
    rhs = (degree + 1) * np.log(_kappa(theta))
    ok = (deg + 1) * lhs <= rhs * (1 - 1e-12)          # criterion holds at d
    prev = (deg * lhs) <= rhs * (1 + 1e-12)            # and fails at d - 1
    assert np.all((deg >= deg_min) & (deg <= degree))
    assert np.all(ok | (deg == degree))
    assert not np.any(prev & (deg > deg_min))
    assert 0 < np.mean(deg < degree) < 1                # the rule is exercised


def test_rule_off_is_fixed_degree(orc):
    src = inputs.points("uniform", 3000, 5)
    w = inputs.weights(3000, 5)
    L = orc.lists(src, 100, src, 0.7, 64, 32, 512, degree=6, deg_min=0)
    assert np.all(L["prox_deg"] == 6)
    a = orc.treecode("stokeslet", src, src, w, 0.01, 6, 0.7, 100, mac_mode=1, order_leaf=32)
    b = orc.treecode("stokeslet", src, src, w, 0.01, 6, 0.7, 100, mac_mode=1, order_leaf=32,
                     deg_min=6)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]


@pytest.mark.parametrize("mode", [0, 1])
def test_rule_poly_exact(orc, mode):
    """(c + x.y)^p with p <= deg_min is reproduced by every cluster's own
    degree, so the treecode equals the direct sum; a cluster evaluated with
    another degree's grid or weights would break this."""
    pts = inputs.points("uniform", 3000, 21)
    w = inputs.weights(3000, 21)
    d = orc.direct("poly", pts, pts, w, poly_p=3, poly_c=1.5)
    t, npx, _ = orc.treecode("poly", pts, pts, w, 0.0, 9, 0.8, 100, mac_mode=mode,
                             order_leaf=32, poly_p=3, poly_c=1.5, deg_min=3)
    t9, npx9, _ = orc.treecode("poly", pts, pts, w, 0.0, 9, 0.8, 100, mac_mode=mode,
                               order_leaf=32, poly_p=3, poly_c=1.5)
    assert 0 < npx < npx9
    assert orc.rel_l2(d, t) < 1e-12
    t4, _, _ = orc.treecode("poly", pts, pts, w, 0.0, 4, 0.8, 100, mac_mode=mode,
                            order_leaf=32, poly_p=3, poly_c=1.5, deg_min=3)
    assert orc.rel_l2(d, t4) < 1e-12
    # clusters the rule puts below the polynomial degree are inexact
    t2, _, _ = orc.treecode("poly", pts, pts, w, 0.0, 4, 0.8, 100, mac_mode=mode,
                            order_leaf=32, poly_p=3, poly_c=1.5, deg_min=1)
    assert orc.rel_l2(d, t2) > 1e-10


def test_rule_counts_and_convergence(orc):
    src = inputs.points("uniform", 6000, 12)
    w = inputs.weights(6000, 12)
    d = orc.direct("stokeslet", src, src, w, eps=0.01)
    L = orc.lists(src, 150, src, 0.7, 64, 32, 512, degree=8, deg_min=1)
    out, npx, _ = orc.treecode("stokeslet", src, src, w, 0.01, 8, 0.7, 150, mac_mode=1,
                               order_leaf=32, deg_min=1)
    cnt = np.diff(L["bptr"])
    b = np.repeat(np.arange(cnt.size), np.diff(L["prox_ptr"]))
    assert npx == int(np.sum(cnt[b] * (L["prox_deg"] + 1) ** 3))
    errs = [orc.rel_l2(d, orc.treecode("stokeslet", src, src, w, 0.01, n, 0.7, 150,
                                       mac_mode=1, order_leaf=32, deg_min=1)[0])
            for n in (4, 6, 8, 10)]
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6
