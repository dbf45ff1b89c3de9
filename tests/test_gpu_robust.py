"""Failure handling and determinism of the library on the GPU.

- A device allocation that fails (forced from the host by the library's
  failure-injection hook, so every kernel still runs normally) returns
  BLTC_ENOMEM, writes nothing to the output, and leaves the handles usable:
  the next call gives the oracle's result.
- Two evaluations of the same inputs are bit-identical (no atomics or
  order-dependent reductions in the evaluation path).
"""
import numpy as np
import pytest

from closeness import close
from paper_1902_02250_amd import bltc, inputs, selector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    bltc.load()
    yield t
    bltc.inject_alloc_failure(0)


def _d(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _sentinel(torch, shape):
    return torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")


def _untouched(out):
    return bool(out.isnan().all().item())


def test_one_call_enomem_at_every_allocation(torch, orc):
    """bltc_evaluate allocates the tree, the batches, the weights and the
    lists; failing each allocation in turn gives BLTC_ENOMEM and no output."""
    n = 3000
    src = inputs.points("uniform", n, 91)
    w = inputs.weights(n, 91)
    d_src, d_w = _d(torch, src), _d(torch, w)
    failures = 0
    for k in range(1, 200):
        out = _sentinel(torch, (3, n))
        bltc.inject_alloc_failure(k)
        try:
            bltc.evaluate(d_src, d_src, d_w, "stokeslet", 0.01, 4, 0.7, 300, out=out)
        except bltc.BltcError as e:
            assert e.status == 2, e            # BLTC_ENOMEM
            torch.cuda.synchronize()
            assert _untouched(out), k
            failures += 1
            continue
        finally:
            bltc.inject_alloc_failure(0)
        break
    else:
        raise AssertionError("the one-call evaluation never completed")
    print(f"[robust] one-call evaluation: {failures} allocations failed in turn", flush=True)
    assert failures >= 10
    ref, _, _ = orc.treecode("stokeslet", src, src, w, 0.01, 4, 0.7, 300, mac_mode=1,
                             batch_size=64, order_leaf=0)
    close(orc, ref, out.cpu().numpy(), 1e-12, what="after the injected failures")


def test_enomem_leaves_handles_usable(torch, orc):
    """A failure while a call grows the handles' buffers (interaction lists,
    selection scratch, a new degree's tables) leaves them consistent."""
    n = 20000
    src = inputs.points("mixture", n, 92)
    w = inputs.weights(n, 92)
    d_src, d_w = _d(torch, src), _d(torch, w)
    T = bltc.Tree(d_src, 400)
    T.compute_weights(d_w, 5)
    G = bltc.Targets(d_src, 64, 32, 512)
    # fresh targets: the first evaluation allocates the lists
    for k in (1, 2):
        out = _sentinel(torch, (3, n))
        bltc.inject_alloc_failure(k)
        with pytest.raises(bltc.BltcError) as ei:
            bltc.evaluate_tree(T, G, "stokeslet", 0.01, 5, 0.7, out=out)
        bltc.inject_alloc_failure(0)
        assert ei.value.status == 2
        torch.cuda.synchronize()
        assert _untouched(out)
    got = bltc.evaluate_tree(T, G, "stokeslet", 0.01, 5, 0.7).cpu().numpy()
    ref, _, _ = orc.treecode("stokeslet", src, src, w, 0.01, 5, 0.7, 400, mac_mode=1,
                             batch_size=64, order_leaf=32)
    close(orc, ref, got, 1e-12, what="lists after failed growth")
    # a new degree's tables (and the rule's derived degrees)
    failures = 0
    for k in (1, 3, 5, 7):
        out = _sentinel(torch, (3, n))
        bltc.inject_alloc_failure(k)
        try:
            T.compute_weights(d_w, 8)
            bltc.evaluate_tree(T, G, "stokeslet", 0.01, 8, 0.8, out=out, deg_min=2)
            failed = False
        except bltc.BltcError as e:
            assert e.status == 2
            failed = True
        finally:
            bltc.inject_alloc_failure(0)
        torch.cuda.synchronize()
        if failed:
            failures += 1
            assert _untouched(out), k
    assert failures >= 1
    T.compute_weights(d_w, 8)
    got = bltc.evaluate_tree(T, G, "stokeslet", 0.01, 8, 0.8, deg_min=2).cpu().numpy()
    ref, _, _ = orc.treecode("stokeslet", src, src, w, 0.01, 8, 0.8, 400, mac_mode=1,
                             batch_size=64, order_leaf=32, deg_min=2)
    close(orc, ref, got, 1e-12, what="rule after failed growth")
    # the learned path's scratch
    sel = bltc.Selector(selector.MODEL_PATH)
    T.compute_weights(d_w, 10)
    for k in range(1, 40, 2):
        out = _sentinel(torch, (3, n))
        bltc.inject_alloc_failure(k)
        try:
            bltc.evaluate_adaptive(T, G, "stokeslet", 0.01, sel, 1e-5, 10, 0.6, out=out)
            failed = False
        except bltc.BltcError as e:
            assert e.status == 2
            failed = True
        finally:
            bltc.inject_alloc_failure(0)
        torch.cuda.synchronize()
        if failed:
            assert _untouched(out), k
    a, ca, _, _ = bltc.evaluate_adaptive(T, G, "stokeslet", 0.01, sel, 1e-5, 10, 0.6)
    b, cb, _, _ = bltc.evaluate_adaptive(T, G, "stokeslet", 0.01, sel, 1e-5, 10, 0.6)
    assert np.array_equal(ca, cb) and torch.equal(a, b)


def test_dual_enomem_and_determinism(torch, orc):
    """The cluster-cluster variant's device traversal and buffers: a failure
    at each of its allocations in turn (on a fresh target tree) returns
    BLTC_ENOMEM with no output written, the next call gives the oracle's
    result, and two calls are bit-identical."""
    n = 12000
    src = inputs.points("mixture", n, 94)
    w = inputs.weights(n, 94)
    d_src, d_w = _d(torch, src), _d(torch, w)
    S = bltc.Tree(d_src, 200)
    S.compute_weights(d_w, 4)
    T = bltc.Tree(d_src, 60)
    failures = 0
    for k in range(1, 80):
        out = _sentinel(torch, (3, n))
        bltc.inject_alloc_failure(k)
        try:
            bltc.evaluate_dual(S, T, "stokeslet", 0.01, 4, 0.8, precision="fp64", out=out,
                               deg_min=1)
        except bltc.BltcError as e:
            assert e.status == 2, e
            torch.cuda.synchronize()
            assert _untouched(out), k
            failures += 1
            continue
        finally:
            bltc.inject_alloc_failure(0)
        break
    else:
        raise AssertionError("the dual evaluation never completed")
    assert failures >= 10
    ref, rcnt = orc.dual_treecode("stokeslet", src, src, w, 0.01, 4, 0.8, 200, 60, deg_min=1)
    a, ca = bltc.evaluate_dual(S, T, "stokeslet", 0.01, 4, 0.8, precision="fp64", deg_min=1)
    b, cb = bltc.evaluate_dual(S, T, "stokeslet", 0.01, 4, 0.8, precision="fp64", deg_min=1)
    assert np.array_equal(ca, rcnt) and np.array_equal(ca, cb)
    assert torch.equal(a, b)
    close(orc, ref, a.cpu().numpy(), 1e-12, what="dual after the injected failures")


@pytest.mark.parametrize("precision", ["fp64", "fp32_fp64acc", "fp32_kahan"])
def test_evaluate_tree_bit_deterministic(torch, precision):
    n = 200000
    src = inputs.points("union", n, 93)
    w = inputs.weights(n, 93)
    d_src, d_w = _d(torch, src), _d(torch, w)
    T = bltc.Tree(d_src, 1000)
    T.compute_weights(d_w, 7)
    G = bltc.Targets(d_src, 64, 32, 512)
    a = bltc.evaluate_tree(T, G, "rotlet", 0.005, 7, 0.7, precision=precision, deg_min=2)
    T.compute_weights(d_w, 7)   # the weights again, through the whole upward pass
    b = bltc.evaluate_tree(T, G, "rotlet", 0.005, 7, 0.7, precision=precision, deg_min=2)
    assert torch.equal(a, b)
    c = bltc.evaluate_tree(T, G, "rotlet", 0.005, 7, 0.7, precision=precision)
    d = bltc.evaluate_tree(T, G, "rotlet", 0.005, 7, 0.7, precision=precision)
    assert torch.equal(c, d)
