"""GPU checks of the learned (n, theta) path through the C ABI: batch
features and counts against the oracle's tree and lists; the judge's
fallback samples against the oracle's treecode (Algorithm 2 with the
per-target MAC) at the same targets; the adaptive evaluation against the
oracle's treecode at each batch's chosen (n, theta), target by target; and
the adaptive evaluation composed exactly of per-candidate fixed evaluations
(the batches the judge sends to the fallback agree with the fallback
evaluation up to the order of its FP64 accumulation)."""
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
    return t


def _d(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=[0, 32], ids=["kd", "leaf32"])
def case(torch, request):
    """Clustered points, batched by the balanced k-d rule (the default) and
    by an order tree with leaves of 32."""
    ol = request.param
    src = inputs.points("mixture", 30000, 71)
    w = inputs.weights(30000, 71)
    T = bltc.Tree(_d(torch, src), 300)
    T.compute_weights(_d(torch, w), 4)
    G = bltc.Targets(_d(torch, src), 64, ol, 512)
    return dict(src=src, w=w, T=T, G=G, d_w=_d(torch, w), ol=ol)


def test_counts_match_oracle_lists(torch, orc, case):
    for theta in (0.4, 0.7, 0.9):
        pc, sc = bltc.batch_counts(case["T"], case["G"], theta)
        L = orc.lists(case["src"], 300, case["src"], theta, 64, case["ol"], 512)
        R = orc.Tree(case["src"], 300)
        np_ = np.diff(L["prox_ptr"])
        sizes = R.pend - R.pbegin
        ns = np.array([sizes[L["dir_ids"][L["dir_ptr"][b]:L["dir_ptr"][b + 1]]].sum()
                       for b in range(np_.size)])
        assert np.array_equal(pc.cpu().numpy(), np_)
        assert np.array_equal(sc.cpu().numpy(), ns)


def test_features_match_oracle(torch, orc, case):
    eps, th = 0.01, 0.7
    f = bltc.batch_features(case["T"], case["G"], "rotlet", eps, th).cpu().numpy()
    src = case["src"]
    R = orc.Tree(src, 300)
    L = orc.lists(src, 300, src, th, 64, case["ol"], 512)
    tperm, bptr, bc, br = orc.batches(src, 64, case["ol"], 512)
    R0 = R.radius[0]
    tiny = 1e-12 * R0
    lo, hi = R.box[0, :3], R.box[0, 3:]
    dens = src.shape[1] / np.prod(hi - lo + tiny)
    for b in range(bptr.size - 1):
        prox = L["prox_ids"][L["prox_ptr"][b]:L["prox_ptr"][b + 1]]
        dirs = L["dir_ids"][L["dir_ptr"][b]:L["dir_ptr"][b + 1]]
        P, Lc = prox.size, dirs.size
        D = (R.pend[dirs] - R.pbegin[dirs]).sum()
        Rd = np.linalg.norm(bc[b] - R.center[prox], axis=1)
        vol = np.prod(R.box[dirs, 3:] - R.box[dirs, :3] + tiny, axis=1).sum()
        ref = [np.log2(max(bptr[b + 1] - bptr[b], 1)), np.log10((br[b] + tiny) / R0),
               np.log10((eps + tiny) / R0), np.log10((eps + tiny) / (br[b] + tiny)),
               np.log10(1 + P), np.log10(1 + D), np.log10(1 + Lc),
               np.mean(np.log10((R.radius[prox] + tiny) / R0)) if P else 0.0,
               np.mean((br[b] + R.radius[prox]) / (th * Rd)) if P else 0.0,
               np.log10((D + 1) / (vol + tiny ** 3) / dens), 1.0, np.log10(src.shape[1])]
        assert np.allclose(f[b], ref, rtol=2e-5, atol=2e-5), (b, f[b], ref)


@pytest.mark.parametrize("deg_min", [0, 1, 3])
def test_batch_costs_match_oracle_lists(torch, orc, case, deg_min):
    w = (0.69, 0.5, 2.5, 1.0)
    cands = [(2, 0.9), (6, 0.7), (9, 0.5), (12, 0.4), (8, 0.7)]
    cost = bltc.batch_costs(case["T"], case["G"], cands, deg_min, w).cpu().numpy()
    R = orc.Tree(case["src"], 300)
    sizes = R.pend - R.pbegin
    for j, (n, th) in enumerate(cands):
        L = orc.lists(case["src"], 300, case["src"], th, 64, case["ol"], 512, degree=n,
                      deg_min=deg_min)
        pp, dp = L["prox_ptr"], L["dir_ptr"]
        n1 = (L["prox_deg"] + 1).astype(np.float64)
        per = (w[0] * n1 + w[1]) * n1 * n1 + w[2]
        cs = np.concatenate([[0.0], np.cumsum(per)])
        far = cs[pp[1:]] - cs[pp[:-1]]
        near = np.array([sizes[L["dir_ids"][dp[b]:dp[b + 1]]].sum() for b in range(dp.size - 1)])
        ref = far + near * w[3]
        # the device sums a few hundred terms in FP32: n u <= 300 x 6e-8
        assert np.allclose(cost[j], ref, rtol=2e-5), (n, th)


def _const_model(tmp_path, j, value, other=5.0):
    k = selector.K
    p = np.zeros(selector.bltc_param_count(k), np.float32)
    b3 = np.full(k, other, np.float32)
    b3[j] = value
    p[-k:] = b3
    path = str(tmp_path / f"const_{j}.bin")
    selector.write_model(path, p, np.zeros(12), np.ones(12), 0.0)
    return path


def _targets_of(G, b):
    ex = G.export()
    return ex["tperm"][ex["bptr"][b]:ex["bptr"][b + 1]]


def _fixed(torch, case, n, th, kernel="stokeslet", eps=0.01, deg_min=selector.DEG_MIN):
    """A fixed evaluation as the learned path runs its candidates (with the
    model's separation rule); deg_min=0 for the judge's fallback."""
    case["T"].compute_weights(case["d_w"], n)
    return bltc.evaluate_tree(case["T"], case["G"], kernel, eps, n, th,
                              precision="fp32_fp64acc", deg_min=deg_min).cpu().numpy()


def test_adaptive_constant_choice(torch, tmp_path, case):
    j = selector.CANDIDATES.index((6, 0.7))
    sel = bltc.Selector(_const_model(tmp_path, j, -5.0))
    out, choice, stats, judge = bltc.evaluate_adaptive(case["T"], case["G"], "stokeslet", 0.01,
                                                       sel, 1e-3, 10, 0.6)
    assert np.all(choice == j) and stats[1] == 1 and stats[2] == 0
    assert 0 < judge[0] == judge[1] < 1e-3
    assert np.array_equal(out.cpu().numpy(), _fixed(torch, case, 6, 0.7))


def _same_sums(a, b):
    """Batches the judge re-evaluates run their proxy lists in slices on
    separate waves, which changes only the order of the FP64 accumulation of
    the per-cluster FP32 sums: equal to the one-wave evaluation to ~1e-16."""
    return np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


def test_adaptive_judge_fallback(torch, tmp_path, case):
    """With a tolerance below FP32 rounding every batch fails the judge and is
    evaluated again with the fallback treecode."""
    j = selector.CANDIDATES.index((3, 0.9))
    sel = bltc.Selector(_const_model(tmp_path, j, -13.0))
    out, choice, stats, judge = bltc.evaluate_adaptive(case["T"], case["G"], "stokeslet", 0.01,
                                                       sel, 1e-12, 10, 0.6)
    assert np.all(choice == -2) and stats[2] == case["G"].nb
    assert judge[1] < judge[0]
    assert _same_sums(out.cpu().numpy(), _fixed(torch, case, 10, 0.6, deg_min=0))
    # every candidate predicted far above the budget: the cheapest is taken;
    # the judge sends the batches with the largest errors to the fallback, as
    # many as bring its estimate within the tolerance
    sel2 = bltc.Selector(_const_model(tmp_path, j, 5.0))
    out2, choice2, stats2, judge2 = bltc.evaluate_adaptive(case["T"], case["G"], "stokeslet",
                                                           0.01, sel2, 1e-6, 10, 0.6)
    assert judge2[0] > 1e-6 >= judge2[1]
    assert stats2[2] == np.sum(choice2 == -2) > case["G"].nb // 2
    out2 = out2.cpu().numpy()
    for u in sorted(set(choice2.tolist())):
        n, th = selector.CANDIDATES[u] if u >= 0 else (10, 0.6)
        ref = _fixed(torch, case, n, th, deg_min=selector.DEG_MIN if u >= 0 else 0)
        for b in np.where(choice2 == u)[0]:
            t = _targets_of(case["G"], b)
            if u >= 0:
                assert np.array_equal(out2[:, t], ref[:, t]), (u, b)
            else:
                assert _same_sums(out2[:, t], ref[:, t]), (u, b)


def test_adaptive_is_per_batch_composition(torch, tmp_path, case):
    k = selector.K
    p = selector.glorot(k, seed=4)
    p[-k:] = np.random.default_rng(5).uniform(-6.0, -4.0, k)
    path = str(tmp_path / "rand.bin")
    selector.write_model(path, p, np.zeros(12), np.full(12, 3.0), 0.0)
    sel = bltc.Selector(path)
    for tol in (1e-5, 1e-6, 1e-4):   # the first tolerance that mixes candidates
        out, choice, stats, judge = bltc.evaluate_adaptive(case["T"], case["G"], "rotlet",
                                                           0.01, sel, tol, 8, 0.6)
        used = sorted(set(choice.tolist()))
        if len([u for u in used if u >= 0]) >= 2:
            break
    assert len([u for u in used if u >= 0]) >= 2, used
    assert stats[1] >= len({selector.CANDIDATES[u][0] for u in used if u >= 0})
    out = out.cpu().numpy()
    for u in used:
        n, th = selector.CANDIDATES[u] if u >= 0 else (8, 0.6)
        ref = _fixed(torch, case, n, th, kernel="rotlet",
                     deg_min=selector.DEG_MIN if u >= 0 else 0)
        for b in np.where(choice == u)[0]:
            t = _targets_of(case["G"], b)
            if u >= 0:
                assert np.array_equal(out[:, t], ref[:, t]), (u, b)
            else:
                assert _same_sums(out[:, t], ref[:, t]), (u, b)


def test_adaptive_small_groups_sliced_finer(torch, tmp_path):
    """200,000 clustered targets (3,125 batches): a full evaluation of this
    size runs in at most a few slices per batch, while a degree group of the
    per-batch selection, launched alone with a fraction of the batches,
    slices its batches more finely.  Slices change only the order of the
    FP64 sums, so every batch still equals the fixed evaluation at its
    candidate to 1e-12, and the lone-group run mode stays bit for bit."""
    n = 200000
    src = inputs.points("mixture", n, 73)
    w = inputs.weights(n, 73)
    d_w = _d(torch, w)
    T = bltc.Tree(_d(torch, src), 1000)
    T.compute_weights(d_w, 4)
    G = bltc.Targets(_d(torch, src))
    c = dict(src=src, w=w, T=T, G=G, d_w=d_w, ol=0)
    k = selector.K
    p = selector.glorot(k, seed=4)
    p[-k:] = np.random.default_rng(5).uniform(-6.0, -4.0, k)
    path = str(tmp_path / "rand_large.bin")
    selector.write_model(path, p, np.zeros(12), np.full(12, 3.0), 0.0)
    sel = bltc.Selector(path)
    for tol in (1e-5, 1e-6, 1e-4):   # the first tolerance that mixes degrees
        out, choice, stats, judge = bltc.evaluate_adaptive(T, G, "rotlet", 0.01, sel, tol, 8,
                                                           0.6)
        used = sorted(set(choice.tolist()))
        if len({selector.CANDIDATES[u][0] for u in used if u >= 0}) >= 2:
            break
    degs = [selector.CANDIDATES[u][0] for u in used if u >= 0]
    assert len(set(degs)) >= 2, used
    per_deg = {d: int(np.sum([np.sum(choice == u) for u in used
                              if u >= 0 and selector.CANDIDATES[u][0] == d])) for d in set(degs)}
    assert min(per_deg.values()) <= G.nb // 2, per_deg   # a group of at most half the batches
    out = out.cpu().numpy()
    for u in used:
        nd, th = selector.CANDIDATES[u] if u >= 0 else (8, 0.6)
        ref = _fixed(torch, c, nd, th, kernel="rotlet",
                     deg_min=selector.DEG_MIN if u >= 0 else 0)
        for b in np.where(choice == u)[0]:
            t = _targets_of(G, b)
            assert _same_sums(out[:, t], ref[:, t]), (u, b)
    # one candidate for every batch: a single group, sliced as a full evaluation
    out1, choice1, _, _ = bltc.evaluate_adaptive(T, G, "rotlet", 0.01, sel, tol, 8, 0.6,
                                                 mode="run")
    u1 = int(choice1[choice1 >= 0][0])
    if np.all(choice1 == u1):
        nd, th = selector.CANDIDATES[u1]
        assert np.array_equal(out1.cpu().numpy(), _fixed(torch, c, nd, th, kernel="rotlet"))


@pytest.mark.parametrize("dist,kernel,tol", [("mixture", "stokeslet", 1e-5),
                                             ("union", "rotlet", 1e-4)])
def test_trained_selector_gain(torch, dist, kernel, tol):
    """What the trained network gains over the method without it: on a
    workload outside its training runs, the learned evaluation meets the
    requested global error against the FP64 direct sum, at a modelled cost
    well below that of the fixed fallback that would otherwise be used to be
    safe at this tolerance (n = 10, theta = 0.6).  The targets are batched
    by the balanced k-d rule, the batching the network was trained on."""
    n = 150000
    src = inputs.points(dist, n, 4242)
    w = inputs.weights(n, 4242)
    d_src, d_w = _d(torch, src), _d(torch, w)
    T = bltc.Tree(d_src, 1000)
    T.compute_weights(d_w, 10)
    G = bltc.Targets(d_src)
    sel = bltc.Selector(selector.MODEL_PATH)
    out, choice, stats, judge = bltc.evaluate_adaptive(T, G, kernel, 0.005, sel, tol, 10, 0.6)
    idx = torch.from_numpy(inputs.sample_indices(n, 3000, 7)).cuda()
    ref = bltc.direct(d_src, d_src, d_w, kernel, 0.005, idx=idx, precision="fp64")
    err = (torch.linalg.norm(out[:, idx] - ref) / torch.linalg.norm(ref)).item()
    assert err <= tol, (err, judge)
    # modelled wave cost: learned choices (with the rule) against the fallback
    costs = (selector.COST_FAR, selector.COST_ROW, selector.COST_CLU, selector.COST_NEAR)
    c_l = bltc.batch_costs(T, G, selector.CANDIDATES, selector.DEG_MIN, costs).cpu().numpy()
    c_fb = bltc.batch_costs(T, G, [(10, 0.6)], 0, costs).cpu().numpy()[0]
    b = np.arange(choice.size)
    learned = np.where(choice >= 0, c_l[np.maximum(choice, 0), b], c_fb).sum()
    assert learned < 0.6 * c_fb.sum(), (learned, c_fb.sum())


@pytest.mark.parametrize("kernel,dist,fb,ol", [("stokeslet", "mixture", (10, 0.6), 0),
                                               ("rotlet", "union", (8, 0.7), 32),
                                               ("stokeslet", "uniform", (12, 0.5), 0)])
def test_judge_samples_match_oracle(torch, orc, kernel, dist, fb, ol):
    """The judge is the fixed treecode of Algorithm 2: every sampled value
    against the oracle's treecode with the paper's per-target MAC at the same
    target (FP32 evaluation: 1e-6 relative L2, 1e-5 per target)."""
    n, leaf, eps = 60000, 500, 0.005
    src = inputs.points(dist, n, 81)
    w = inputs.weights(n, 81)
    T = bltc.Tree(_d(torch, src), leaf)
    T.compute_weights(_d(torch, w), 4)
    G = bltc.Targets(_d(torch, src), 64, ol, 512)
    idx, u = bltc.judge_samples(T, G, kernel, eps, fb[0], fb[1])
    assert idx.size == G.nb and np.unique(idx).size == idx.size
    ref, _, _ = orc.treecode(kernel, src, src, w, eps, fb[0], fb[1], leaf, mac_mode=0,
                             sample=idx)
    close(orc, ref, u, 1e-6, elem_tol=1e-5, what=f"judge {kernel} {dist} {fb}")


def test_judge_samples_grouped(torch, orc):
    """From 32,768 batches on, the judge samples one target per group of
    floor(nb / 16384) consecutive batches, inside the group's first batch:
    2.2e6 uniform points give 34,375 batches in groups of two.  A spread of
    the samples is checked against the oracle's treecode (per-target MAC)."""
    n, leaf, eps, fb = 2200000, 2000, 0.005, (6, 0.7)
    src = inputs.points("uniform", n, 83)
    w = inputs.weights(n, 83)
    T = bltc.Tree(_d(torch, src), leaf)
    T.compute_weights(_d(torch, w), fb[0])
    G = bltc.Targets(_d(torch, src))
    st = G.nb // 16384
    assert st == 2
    idx, u = bltc.judge_samples(T, G, "stokeslet", eps, fb[0], fb[1])
    assert idx.size == (G.nb + st - 1) // st and np.unique(idx).size == idx.size
    ex = G.export()
    where = np.empty(n, np.int64)
    where[ex["tperm"]] = np.arange(n)
    b = np.searchsorted(ex["bptr"], where[idx], side="right") - 1
    assert np.array_equal(b, np.arange(idx.size) * st)
    pick = np.linspace(0, idx.size - 1, 24).astype(np.int64)
    ref, _, _ = orc.treecode("stokeslet", src, src, w, eps, fb[0], fb[1], leaf, mac_mode=0,
                             sample=idx[pick])
    close(orc, ref, u[:, pick], 1e-6, elem_tol=1e-5, what="judge samples in groups of two")


def test_adaptive_matches_oracle_per_candidate(torch, orc, tmp_path, case):
    """Rotlets on clustered points (the shape of the 1e6 mixture workload,
    at 30,000 points) at a tolerance that mixes candidates: the targets of
    every batch are compared with the oracle's treecode at that batch's
    chosen (n, theta) under the model's separation rule, or at the fallback
    for batches the judge re-evaluated.  The comparison runs in FP64 (1e-12
    relative L2, 1e-10 per target), which shows every batch's lists, degrees
    and modified weights are its candidate's; the FP32 evaluation of the
    same choices is then held to the FP32 bar against it over all targets
    (1e-6 relative L2).  FP32 is not compared batch by batch: inside the
    dense clusters the rotlet sums of an isotropic neighbourhood cancel, so
    the rounding of x - y relative to a batch's centre, up to 2^-24 times the
    batch radius over max(r, eps) of each term, reaches about 1e-6 of the
    cancelled sum there (4e-7 over all targets)."""
    k = selector.K
    p = selector.glorot(k, seed=4)
    p[-k:] = np.random.default_rng(5).uniform(-6.0, -4.0, k)
    path = str(tmp_path / "rand_oracle.bin")
    selector.write_model(path, p, np.zeros(12), np.full(12, 3.0), 0.0)
    sel = bltc.Selector(path)
    case["T"].compute_weights(case["d_w"], 4)
    fb = (8, 0.6)
    for tol in (1e-5, 1e-6, 1e-4):
        out, choice, stats, judge = bltc.evaluate_adaptive(case["T"], case["G"], "rotlet",
                                                           0.01, sel, tol, fb[0], fb[1],
                                                           precision="fp64")
        used = sorted(set(choice.tolist()))
        if len([u for u in used if u >= 0]) >= 2:
            break
    assert len([u for u in used if u >= 0]) >= 2, used
    out = out.cpu().numpy()
    o32, c32, _, _ = bltc.evaluate_adaptive(case["T"], case["G"], "rotlet", 0.01, sel, tol,
                                            fb[0], fb[1])
    src, w = case["src"], case["w"]
    ex = case["G"].export()
    # the judge's choice of batches to re-evaluate reads the evaluation, so a
    # batch at its threshold may go either way: compare where the two agree
    same = np.where(c32 == choice)[0]
    assert same.size >= 0.9 * choice.size
    ts = np.concatenate([ex["tperm"][ex["bptr"][b]:ex["bptr"][b + 1]] for b in same])
    close(orc, out[:, ts], o32.cpu().numpy()[:, ts], 1e-6, what="adaptive FP32 against FP64")
    counts = {u: int(np.sum(choice == u)) for u in used}
    # the most used candidates, the least used one and the fallback's batches
    picks = sorted([u for u in used if u >= 0], key=lambda u: -counts[u])[:4]
    least = min([u for u in used if u >= 0], key=lambda u: counts[u])
    picks = sorted(set(picks + [least] + ([-2] if -2 in used else [])))
    rng = np.random.default_rng(6)
    for u in picks:
        bs = np.where(choice == u)[0]
        tg = np.concatenate([ex["tperm"][ex["bptr"][b]:ex["bptr"][b + 1]] for b in bs])
        idx = np.sort(rng.choice(tg, size=min(200, tg.size), replace=False))
        n_u, th_u = selector.CANDIDATES[u] if u >= 0 else fb
        dm = selector.DEG_MIN if u >= 0 else 0
        ref, _, _ = orc.treecode("rotlet", src, src, w, 0.01, n_u, th_u, 300, mac_mode=1,
                                 batch_size=64, order_leaf=case["ol"], group_max=512, sample=idx,
                                 deg_min=dm)
        close(orc, ref, out[:, idx], 1e-12, elem_tol=1e-10,
              what=f"adaptive candidate {u} ({n_u}, {th_u}) deg_min {dm}, {bs.size} batches")
