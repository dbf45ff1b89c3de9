"""Pins of the oracle's cluster tree (Section 6) and target batches.

The tree rules determine the tree uniquely, so checking every rule on every
node pins it: tight boxes, the split/leaf decision, the bisected axes
(side > l_max/sqrt(2)), the midpoint partition, child code order, dropped
empty children, breadth-first numbering and the stable particle order.
"""
import numpy as np
import pytest

from paper_1902_02250_amd import inputs


def _check_tree(T, pts, leaf_max):
    n = pts.shape[1]
    assert sorted(T.perm.tolist()) == list(range(n))
    assert T.pbegin[0] == 0 and T.pend[0] == n
    nn = T.nnodes
    # breadth-first numbering: levels never decrease
    assert np.all(np.diff(T.level) >= 0)
    for q in range(nn):
        idx = T.perm[T.pbegin[q]:T.pend[q]]
        assert idx.size > 0
        # stable partitions of the identity leave every leaf in input order
        if T.child_count[q] == 0:
            assert np.all(np.diff(idx) > 0)
        p = pts[:, idx]
        lo, hi = p.min(axis=1), p.max(axis=1)
        assert np.array_equal(T.box[q, :3], lo) and np.array_equal(T.box[q, 3:], hi)
        assert np.array_equal(T.center[q], 0.5 * (lo + hi))
        h = 0.5 * (hi - lo)
        assert T.radius[q] == np.sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2])
        side = hi - lo
        lmax = side.max()
        cc, cf = T.child_count[q], T.child_first[q]
        if idx.size <= leaf_max or lmax == 0.0:
            assert cc == 0
            continue
        split = side > lmax * np.sqrt(0.5)
        mid = 0.5 * (lo + hi)
        code = np.zeros(idx.size, np.int64)
        for a in range(3):
            if split[a]:
                code |= (p[a] >= mid[a]).astype(np.int64) << a
        used = np.unique(code)
        if used.size < 2:
            assert cc == 0
            continue
        assert cc == used.size
        start = T.pbegin[q]
        for k, c in enumerate(used):
            ch = cf + k
            assert T.parent[ch] == q and T.level[ch] == T.level[q] + 1
            members = idx[code == c]
            assert T.pbegin[ch] == start
            assert np.array_equal(T.perm[T.pbegin[ch]:T.pend[ch]], members)
            start = T.pend[ch]
        assert start == T.pend[q]
    # every leaf respects the size limit unless it is degenerate
    leaves = np.where(T.child_count == 0)[0]
    assert np.sum(T.pend[leaves] - T.pbegin[leaves]) == n


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 3000, 100), ("mixture", 4000, 60),
                                         ("uniform", 500, 1), ("union", 2000, 30)])
def test_tree_rules(orc, dist, n, leaf):
    pts = inputs.points(dist, n, 11)
    T = orc.Tree(pts, leaf)
    _check_tree(T, pts, leaf)


def test_slab_gets_two_and_four_children(orc):
    """A flat slab is bisected only along its long sides (the rectangular
    boxes of Example 2)."""
    rng = np.random.default_rng(1)
    pts = np.stack([rng.uniform(-8, 8, 4000), rng.uniform(-8, 8, 4000), rng.uniform(0, 0.5, 4000)])
    T = orc.Tree(pts, 200)
    _check_tree(T, pts, 200)
    assert T.child_count[0] == 4
    pts2 = np.stack([rng.uniform(-8, 8, 4000), rng.uniform(0, 1, 4000), rng.uniform(0, 1, 4000)])
    T2 = orc.Tree(pts2, 200)
    assert T2.child_count[0] == 2


def test_degenerate_points(orc):
    pts = np.zeros((3, 50))
    T = orc.Tree(pts, 10)
    assert T.nnodes == 1 and T.radius[0] == 0.0
    pts = np.concatenate([np.zeros((3, 30)), np.ones((3, 30))], axis=1)
    T = orc.Tree(pts, 10)
    _check_tree(T, pts, 10)
    assert T.nnodes == 3
    # two adjacent doubles: the midpoint rounds onto one of them
    a = 1.0
    b = np.nextafter(a, 2.0)
    pts = np.array([[a] * 20 + [b] * 20, [0.0] * 40, [0.0] * 40])
    T = orc.Tree(pts, 5)
    _check_tree(T, pts, 5)


def test_uniform_tree_shape(orc):
    """C1 shape: 8000 uniform points with N0 = 500 give 64 leaves in 2 levels."""
    pts, w, cfg = inputs.workload("c1")
    T = orc.Tree(pts, cfg["leaf"])
    assert T.depth == 2 and T.nnodes == 73
    assert np.sum(T.child_count == 0) == 64


def _groups(T, G):
    """Maximal nodes with at most G targets (or leaves), in tree order."""
    out = []

    def rec(q):
        if T.pend[q] - T.pbegin[q] <= G or T.child_count[q] == 0:
            out.append((T.pbegin[q], T.pend[q]))
            return
        for c in range(T.child_count[q]):
            rec(T.child_first[q] + c)
    rec(0)
    return out


@pytest.mark.parametrize("dist,G", [("uniform", 256), ("mixture", 100), ("uniform", 10 ** 9)])
def test_batches(orc, dist, G):
    pts = inputs.points(dist, 3000, 5)
    tperm, bptr, bc, br = orc.batches(pts, 64, 16, G)
    T = orc.Tree(pts, 16)
    assert np.array_equal(tperm, T.perm)
    # every group is cut into chunks of 64 from its start; no batch spans two
    expect = []
    for b, e in _groups(T, G):
        expect.extend(range(b, e, 64))
    assert np.array_equal(bptr, np.array(expect + [3000]))
    for b in range(bc.shape[0]):
        p = pts[:, tperm[bptr[b]:bptr[b + 1]]]
        lo, hi = p.min(axis=1), p.max(axis=1)
        assert np.array_equal(bc[b], 0.5 * (lo + hi))
        h = 0.5 * (hi - lo)
        assert br[b] == np.sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2])
    if G >= 3000:   # one group: plain chunks of the tree order
        assert np.all(np.diff(bptr)[:-1] == 64)
    # one target per batch: zero radius, center on the target
    tperm1, bptr1, bc1, br1 = orc.batches(pts, 1, 64)
    assert np.all(br1 == 0.0)
    assert np.array_equal(bc1, pts[:, tperm1].T)


def test_batches_bound_the_radius(orc):
    """Groups bound the batch radius: no batch is wider than its group."""
    pts = inputs.points("uniform", 20000, 6)
    _, bptr, _, br = orc.batches(pts, 64, 32, 256)
    _, bptr2, _, br2 = orc.batches(pts, 64, 32, 10 ** 9)
    assert br.max() < 0.5 * br2.max()


def _kd_reference(pts, bs):
    """The balanced k-d rule written out with full sorts: a set larger than
    bs is cut along the longest side of its tight box (first of equal
    sides), the first part taking the bs * floor(ceil(c / bs) / 2) smallest
    by (coordinate, index); smaller sets are batches in increasing index."""
    out = []

    def rec(idx):
        if idx.size <= bs:
            out.append(np.sort(idx))
            return
        p = pts[:, idx]
        side = p.max(axis=1) - p.min(axis=1)
        ax = int(np.argmax(side))            # the first of equal sides
        order = idx[np.lexsort((idx, pts[ax, idx]))]
        left = bs * (((idx.size + bs - 1) // bs) // 2)
        rec(order[:left])
        rec(order[left:])

    rec(np.arange(pts.shape[1]))
    return out


@pytest.mark.parametrize("dist,m,bs", [("uniform", 3000, 64), ("mixture", 2001, 64),
                                       ("union", 777, 10), ("uniform", 64, 64),
                                       ("uniform", 65, 64), ("mixture", 5, 64)])
def test_kd_batches(orc, dist, m, bs):
    pts = inputs.points(dist, m, 8)
    tperm, bptr, bc, br = orc.batches(pts, bs, 0)
    ref = _kd_reference(pts, bs)
    assert bptr.size - 1 == len(ref) == (m + bs - 1) // bs
    for b, r in enumerate(ref):
        assert np.array_equal(tperm[bptr[b]:bptr[b + 1]], r), b
    # full batches except the last
    cnt = np.diff(bptr)
    assert np.all(cnt[:-1] == bs) and 0 < cnt[-1] <= bs
    assert sorted(tperm.tolist()) == list(range(m))
    for b in range(bc.shape[0]):
        p = pts[:, tperm[bptr[b]:bptr[b + 1]]]
        lo, hi = p.min(axis=1), p.max(axis=1)
        assert np.array_equal(bc[b], 0.5 * (lo + hi))
        h = 0.5 * (hi - lo)
        assert br[b] == np.sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2])


def test_kd_batches_ties_and_coincident_points(orc):
    """Equal coordinates (a small integer lattice with repeats, and a set of
    identical points) are ordered by target index."""
    rng = np.random.default_rng(9)
    pts = rng.integers(0, 3, size=(3, 500)).astype(np.float64)
    tperm, bptr, _, _ = orc.batches(pts, 16, 0)
    ref = _kd_reference(pts, 16)
    for b, r in enumerate(ref):
        assert np.array_equal(tperm[bptr[b]:bptr[b + 1]], r), b
    same = np.ones((3, 100))
    tperm, bptr, bc, br = orc.batches(same, 8, 0)
    assert np.array_equal(tperm, np.arange(100)) and np.all(br == 0.0)


def test_kd_batches_are_compact(orc):
    """On uniform points the k-d batches are no wider than the batches of
    the order tree's groups, and they are full."""
    pts = inputs.points("uniform", 20000, 6)
    _, bptr_t, _, br_t = orc.batches(pts, 64, 32, 512)
    _, bptr_k, _, br_k = orc.batches(pts, 64, 0)
    assert bptr_k.size - 1 == 313 < bptr_t.size - 1
    assert br_k.mean() < br_t.mean()
