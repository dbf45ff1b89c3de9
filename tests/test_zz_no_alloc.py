"""The allocation-free evaluation entry point against the allocating one.

bltc_evaluate_tree_noalloc keeps its interaction lists in the library's
fixed device array instead of the targets handle; it must give
bltc_evaluate_tree's result bit for bit (same lists, same kernel), on two
calls in a row, the second with a smaller input, and reject what does not
fit or was not prepared before writing anything."""
import numpy as np
import pytest

from paper_1902_02250_amd import bltc, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    bltc.load()
    return t


def _d(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(torch, dist, n, seed, leaf, degree):
    src = inputs.points(dist, n, seed)
    w = inputs.weights(n, seed)
    d_src, d_w = _d(torch, src), _d(torch, w)
    T = bltc.Tree(d_src, leaf)
    T.compute_weights(d_w, degree)
    G = bltc.Targets(d_src, 64, 32, 512)
    return T, G


def test_noalloc_equals_evaluate_tree_two_calls(torch):
    assert bltc.noalloc_scratch_bytes() == 32 << 20
    # first call: 200,000 uniform targets, FP32 evaluation
    n1 = 200000
    print(f"[noalloc] call 1: uniform n={n1} stokeslet degree 6 theta 0.7 fp32_fp64acc",
          flush=True)
    T1, G1 = _case(torch, "uniform", n1, 61, 1000, 6)
    ref1 = bltc.evaluate_tree(T1, G1, "stokeslet", 0.005, 6, 0.7, precision="fp32_fp64acc")
    out1 = torch.full((3, n1), float("nan"), dtype=torch.float64, device="cuda")
    bltc.evaluate_tree_noalloc(T1, G1, "stokeslet", 0.005, 6, 0.7, out1,
                               precision="fp32_fp64acc")
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    # second call, smaller: 30,000 mixture targets, rotlet in FP64 with the
    # separation rule (its lower degrees derived by the allocating call)
    n2 = 30000
    print(f"[noalloc] call 2: mixture n={n2} rotlet degree 8 theta 0.8 deg_min 2 fp64",
          flush=True)
    T2, G2 = _case(torch, "mixture", n2, 62, 200, 8)
    ref2 = bltc.evaluate_tree(T2, G2, "rotlet", 0.01, 8, 0.8, precision="fp64", deg_min=2)
    out2 = torch.full((6, n2), float("nan"), dtype=torch.float64, device="cuda")
    bltc.evaluate_tree_noalloc(T2, G2, "rotlet", 0.01, 8, 0.8, out2, precision="fp64",
                               deg_min=2)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref2)
    # and the first case again after the smaller one (stale list contents)
    out1b = torch.full((3, n1), float("nan"), dtype=torch.float64, device="cuda")
    bltc.evaluate_tree_noalloc(T1, G1, "stokeslet", 0.005, 6, 0.7, out1b,
                               precision="fp32_fp64acc")
    torch.cuda.synchronize()
    assert torch.equal(out1b, ref1)


def test_noalloc_rejects_before_writing(torch):
    n = 200000
    print(f"[noalloc] rejections: uniform n={n}", flush=True)
    T, G = _case(torch, "uniform", n, 63, 50, 3)
    out = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda")
    # theta = 0: every batch lists every leaf, 3,125 batches x about 4,000
    # leaves, far beyond the fixed array
    with pytest.raises(bltc.BltcError) as ei:
        bltc.evaluate_tree_noalloc(T, G, "stokeslet", 0.01, 3, 0.0, out)
    assert ei.value.status == 1 and "bytes" in ei.value.message
    # a degree whose weights were never computed
    with pytest.raises(bltc.BltcError) as ei:
        bltc.evaluate_tree_noalloc(T, G, "stokeslet", 0.01, 5, 0.7, out)
    assert ei.value.status == 4
    # the rule's lower degrees not derived yet
    T.compute_weights(_d(torch, inputs.weights(n, 63)), 9)
    with pytest.raises(bltc.BltcError) as ei:
        bltc.evaluate_tree_noalloc(T, G, "stokeslet", 0.01, 9, 0.7, out, deg_min=2)
    assert ei.value.status == 4
    torch.cuda.synchronize()
    assert out.isnan().all().item()
