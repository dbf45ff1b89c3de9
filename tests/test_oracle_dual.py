"""Pins of the oracle's cluster-cluster variant (interpolation in both the
target and the source variable, Section 9).

- Polynomial kernel (c + x.y)^p with p <= n: interpolation in either
  variable is exact, so the variant reproduces the direct sum; p = 0 (the
  constant kernel) also shows every (target, source) pair is counted once.
  The cases are sized so that all four interaction types occur.
- theta = 0: no cluster pair is accepted and the variant is the direct sum.
- Stokeslets: the error falls as n grows at fixed theta, and stays within a
  small factor of the particle-cluster treecode's at the same (n, theta).
"""
import numpy as np
import pytest

from paper_1902_02250_amd import inputs


@pytest.mark.parametrize("p,c,n,N", [(0, 1.0, 2, 6000), (2, 0.5, 2, 6000), (3, 1.5, 4, 20000)])
def test_dual_poly_exact(orc, p, c, n, N):
    src = inputs.points("mixture", N, 81)
    tgt = inputs.points("uniform", N - 1000, 82)
    w = inputs.weights(N, 81)
    got, cnt = orc.dual_treecode("poly", tgt, src, w, 0.0, n, 0.8, 40, 40, poly_p=p,
                                 poly_c=c)
    assert np.all(cnt[:4] > 0), cnt            # CC, PC, CP and PP all occur
    ref = orc.direct("poly", tgt, src, w, poly_p=p, poly_c=c)
    assert orc.rel_l2(ref, got) <= 1e-12


def test_dual_theta_zero_is_direct(orc):
    src = inputs.points("union", 3000, 83)
    w = inputs.weights(3000, 83)
    for kernel in ("stokeslet", "rotlet", "full"):
        w = inputs.weights(3000, 83, orc.WDIM[kernel])
        got, cnt = orc.dual_treecode(kernel, src, src, w, 0.01, 3, 0.0, 50, 30)
        assert cnt[0] == cnt[1] == cnt[2] == 0 and cnt[3] == 3000 * 3000
        ref = orc.direct(kernel, src, src, w, eps=0.01)
        assert orc.rel_l2(ref, got) <= 1e-13


def test_dual_stokeslet_converges(orc):
    src = inputs.points("uniform", 30000, 84)
    w = inputs.weights(30000, 84)
    ref = orc.direct("stokeslet", src, src, w, eps=0.01)
    errs = []
    for n in (2, 4, 6):
        got, cnt = orc.dual_treecode("stokeslet", src, src, w, 0.01, n, 0.7, 60, 60)
        assert cnt[0] > 0
        errs.append(orc.rel_l2(ref, got))
        pc, _, _ = orc.treecode("stokeslet", src, src, w, 0.01, n, 0.7, 60)
        assert errs[-1] <= 10 * orc.rel_l2(ref, pc) + 1e-14, (n, errs[-1])
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 1e-5, errs


def test_dual_full_is_sum_of_parts(orc):
    """Six weight rows: the full kernel's result is the Stokeslet result of
    the forces plus the rotlet result of the torques, with the rotlet
    velocity of the forces as the angular velocity's force part."""
    src = inputs.points("mixture", 20000, 85)
    w6 = inputs.weights(20000, 85, 6)
    run = lambda k, w: orc.dual_treecode(k, src, src, w, 0.01, 4, 0.8, 40, 40)
    full, cnt = run("full", w6)
    assert cnt[0] > 0
    sf, _ = run("stokeslet", np.ascontiguousarray(w6[:3]))
    rn, _ = run("rotlet", np.ascontiguousarray(w6[3:]))
    rf, _ = run("rotlet", np.ascontiguousarray(w6[:3]))
    ref = np.concatenate([sf + rn[:3], rf[:3] + rn[3:]])
    assert orc.rel_l2(ref, full) <= 1e-13


def test_dual_rule_poly_exact(orc):
    """Separation rule on the source side: every degree used is at least
    deg_min = p, so (c + x.y)^p stays exact, while the evaluation counts of
    the CC and PC parts fall below those of the fixed degree."""
    src = inputs.points("mixture", 20000, 86)
    tgt = inputs.points("uniform", 19000, 87)
    w = inputs.weights(20000, 86)
    got, cnt = orc.dual_treecode("poly", tgt, src, w, 0.0, 5, 0.8, 40, 40, poly_p=2,
                                 poly_c=0.5, deg_min=2)
    fixed, cnt0 = orc.dual_treecode("poly", tgt, src, w, 0.0, 5, 0.8, 40, 40, poly_p=2,
                                    poly_c=0.5)
    assert cnt[0] > 0 and cnt[1] > 0
    assert cnt[0] < cnt0[0] and cnt[1] < cnt0[1]
    assert cnt[2] == cnt0[2] and cnt[3] == cnt0[3] and cnt[4] == cnt0[4]
    d = orc.direct("poly", tgt, src, w, poly_p=2, poly_c=0.5)
    assert orc.rel_l2(d, got) <= 1e-12
