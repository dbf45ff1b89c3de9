"""CPU checks of the library: it loads, exports every function its header
declares, builds trees and batches bit-identical to the oracle's (its own
host code, shared with nothing), and rejects bad arguments before touching
a device."""
import ctypes

import numpy as np
import pytest

from paper_1902_02250_amd import bltc, inputs

TREE_KEYS = ["perm", "box", "center", "radius", "child_first", "child_count",
             "pbegin", "pend", "level"]


def test_library_exports_every_declared_symbol():
    L = bltc.load()
    names = bltc.declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name
    assert L.bltc_version().startswith(b"bltc")


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 8000, 500), ("uniform", 20011, 2000),
                                         ("mixture", 30000, 100), ("union", 9000, 7),
                                         ("mixture", 5000, 1)])
def test_host_tree_bit_exact(orc, dist, n, leaf):
    p = inputs.points(dist, n, 17)
    a = bltc.host_tree(p, leaf)
    T = orc.Tree(p, leaf)
    assert a["depth"] == T.depth
    for k in TREE_KEYS:
        assert np.array_equal(a[k], getattr(T, k)), k


def test_host_tree_degenerate(orc):
    cases = [np.zeros((3, 40)),
             np.concatenate([np.zeros((3, 30)), np.ones((3, 31))], axis=1),
             np.array([[1.0] * 10 + [np.nextafter(1.0, 2.0)] * 10, [0.0] * 20, [5.0] * 20]),
             np.stack([np.linspace(-1, 1, 300), np.zeros(300), np.zeros(300)]),
             np.zeros((3, 0)), np.array([[0.5], [0.25], [-1.0]])]
    for p in cases:
        a = bltc.host_tree(p, 4)
        T = orc.Tree(p, 4)
        for k in TREE_KEYS:
            assert np.array_equal(a[k], getattr(T, k)), (k, p.shape)


@pytest.mark.parametrize("bs,leaf,group", [(64, 64, 256), (1, 64, 256), (100, 30, 90),
                                            (1024, 200, 10 ** 9), (256, 256, 300), (64, 16, 1),
                                            (64, 0, 512), (1, 0, 512), (1000, 0, 512)])
def test_host_batches_bit_exact(orc, bs, leaf, group):
    p = inputs.points("mixture", 7777, 3)
    b = bltc.host_batches(p, bs, leaf, group)
    ob = orc.batches(p, bs, leaf, group)
    for x, y in zip([b["tperm"], b["bptr"], b["bcenter"], b["bradius"]], ob):
        assert np.array_equal(x, y)


def _status(rc):
    return bltc.STATUS[rc]


def test_argument_validation_before_device_work():
    L = bltc.load()
    o = bltc.options()
    ok = ctypes.byref(o)
    # evaluate with empty sets: every parameter check still applies
    ev = lambda kern, eps, deg, th, leaf=10, opt=ok: L.bltc_evaluate(
        None, None, None, 0, None, None, None, 0, None, kern, eps, deg, th, leaf, opt, None, None)
    assert _status(ev(0, 0.01, 4, 0.7)) == "OK"
    assert _status(ev(7, 0.01, 4, 0.7)) == "EINVAL"
    assert b"kernel" in L.bltc_last_error()
    assert _status(ev(0, -1.0, 4, 0.7)) == "EINVAL"
    assert _status(ev(0, float("nan"), 4, 0.7)) == "EINVAL"
    assert _status(ev(0, 0.01, 0, 0.7)) == "EINVAL"
    assert _status(ev(0, 0.01, 13, 0.7)) == "EINVAL"
    assert _status(ev(0, 0.01, 4, 1.5)) == "EINVAL"
    assert _status(ev(0, 0.01, 4, -0.1)) == "EINVAL"
    assert _status(ev(0, 0.01, 4, 0.7, leaf=0)) == "EINVAL"
    bad = bltc.options()
    bad.size = 4
    assert _status(ev(0, 0.01, 4, 0.7, opt=ctypes.byref(bad))) == "EINVAL"
    poly32 = bltc.options(precision="fp32_fp64acc")
    assert _status(ev(100, 0.0, 4, 0.7, opt=ctypes.byref(poly32))) == "EINVAL"
    big = bltc.options(batch_size=2048)
    assert _status(ev(0, 0.01, 4, 0.7, opt=ctypes.byref(big))) == "EINVAL"
    # NULL output handle, negative and oversized counts, NULL arrays
    assert _status(L.bltc_build_tree(None, None, None, 0, 10, None, None)) == "EINVAL"
    h = ctypes.c_void_p()
    assert _status(L.bltc_build_tree(None, None, None, -1, 10, None, ctypes.byref(h))) == "EINVAL"
    assert _status(L.bltc_build_tree(None, None, None, 1 << 31, 10, None, ctypes.byref(h))) == "EINVAL"
    assert _status(L.bltc_build_tree(None, None, None, 5, 10, None, ctypes.byref(h))) == "EINVAL"
    assert h.value is None
    assert _status(L.bltc_build_targets(None, None, None, 0, 0, 64, 256, None, ctypes.byref(h))) == "EINVAL"
    assert _status(L.bltc_build_targets(None, None, None, 0, 64, 64, 0, None, ctypes.byref(h))) == "EINVAL"
    assert _status(L.bltc_evaluate_tree(None, None, 0, 0.01, 4, 0.7, ok, None, None)) == "EINVAL"
    assert _status(L.bltc_compute_modified_weights(None, None, 3, 4, None)) == "EINVAL"
    assert _status(L.bltc_direct(None, None, None, 0, None, 0, None, None, None, 0, None, 5, 0.0,
                                 ok, None, None)) == "EINVAL"
    assert _status(L.bltc_direct(None, None, None, 0, None, 3, None, None, None, 0, None, 0, 0.0,
                                 ok, None, None)) == "EINVAL"
    assert _status(L.bltc_host_tree(None, None, None, 3, 4, *([None] * 11))) == "EINVAL"
    assert _status(L.bltc_host_batches(None, None, None, 0, 0, 4, 256, *([None] * 5))) == "EINVAL"
    grp0 = bltc.options(group_max=0)
    assert _status(ev(0, 0.01, 4, 0.7, opt=ctypes.byref(grp0))) == "EINVAL"
