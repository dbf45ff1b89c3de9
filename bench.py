#!/usr/bin/env python3
"""Benchmark of the treecode evaluation phase on one MI355X.

Workload (default): 1,000,000 points i.i.d. uniform in [-1, 1]^3, forces
uniform in [-1, 1]^3, regularized Stokeslets with eps = 0.005, degree n = 8,
MAC theta = 0.7, leaf size N0 = 2000, FP32 kernel evaluation with FP64
per-target accumulation; targets = sources.

One step is the evaluation phase on resident device data: weight gather,
cluster grids and modified weights (upward pass), the batch interaction lists
on the device, and the particle-cluster evaluation with the scatter to caller
order.  The source tree and the target order/batches are built once before
timing (their build time is reported in "build_ms").

Printed on stdout: one JSON line.  value = kernel evaluations performed per
second (far-field proxy evaluations plus near-field pair evaluations, summed
over targets).  Also reported: the relative L2 error against the FP64 direct
sum on a 10,000-target sample (the library's GPU direct sum) and on 2,000
targets against the oracle's CPU direct sum, the headline in the other
accumulation modes, the learned (n, theta) against the best fixed settings at
an error target (a sweep of the candidate grid), the per-stage device times
from the library's HIP events, the roofline of the evaluation kernel and the
CPU oracle's rate.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops per kernel evaluation (FMA = 2, rsqrt = 1), from the
# formulas of eq. Velocity_1 and eq. MRS_2 (both parts together for "full").
FLOPS = {"stokeslet": 32, "rotlet": 58, "full": 92}
# MI355X published vector peaks (TFLOP/s).
PEAK = {"fp32": 157.3, "fp64": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_p2p_stokeslet_n1e6_hbm_traffic.md")
COUNTER_FILE = os.path.join(ROOT, "profiles", "k_p2p_stokeslet_n1e6_valu_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1902_02250_amd", "csrc", f)
                  for f in ("k_p2p.hip", "kmath.h")]


def profile_record(path, key, args, cfg):
    """A per-launch figure of the evaluation kernel from a committed rocprofv3
    summary, or None when that summary is for another workload or launch
    configuration, or the kernel sources changed since it was taken."""
    import hashlib
    if (args.workload, cfg["n"], cfg["degree"], args.precision, args.batch_size,
            args.order_leaf) != ("c3", 1000000, 8, "fp32_fp64acc", 64, 0) \
            or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    rec = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in (key, "kernel_source_sha256"):
            k, v = line.split(":", 1)
            rec[k] = v.strip()
    if rec.get("kernel_source_sha256") != h.hexdigest() or key not in rec:
        return None
    return float(rec[key])


def cpu_baseline(cfg, src, w, sample_k, args, osamp, head_at_osamp):
    """The FP64 oracle treecode (tree, Algorithm 1 weights for all sources,
    batch walk for a target sample) timed on the host cores.  The same leg
    evaluates the oracle's FP64 direct sum (eq. N-body) at the osamp targets
    and reports the headline's error against it."""
    import oracle
    from paper_1902_02250_amd import inputs
    oracle._load()
    idx = inputs.sample_indices(src.shape[1], sample_k, cfg["seed"] + 7)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    _, npx, ndr = oracle.treecode(cfg["kernel"], src, src, w, cfg["eps"], cfg["degree"],
                                  cfg["theta"], cfg["leaf"], mac_mode=1,
                                  batch_size=args.batch_size, order_leaf=args.order_leaf,
                                  group_max=args.group_max, sample=idx)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    ref = oracle.direct_subset(cfg["kernel"], src, osamp, src, w, cfg["eps"])
    dt_direct = time.perf_counter() - t1
    e_oracle = float(np.linalg.norm(head_at_osamp - ref) / np.linalg.norm(ref))
    return {"value": (npx + ndr) / dt, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle treecode from scratch (tree, Algorithm 1 weights for all "
                       f"{src.shape[1]} sources, shared-batch walk) evaluated for {sample_k} "
                       f"seeded targets of the same workload: {npx + ndr} kernel evaluations "
                       f"in {dt:.2f} s on {threads} OpenMP threads"),
            "seconds": dt,
            "rel_l2_err_oracle": e_oracle,
            "oracle_direct": (f"oracle FP64 direct sum at {osamp.size} seeded targets "
                              f"({dt_direct:.2f} s): the headline's relative L2 error "
                              f"against it")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--n", type=int, default=None, help="override the point count")
    ap.add_argument("--precision", default="fp32_fp64acc",
                    choices=["fp64", "fp32_fp64acc", "fp32_kahan"])
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--kernel", default=None, choices=["stokeslet", "rotlet", "full"])
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--eps", type=float, default=None,
                    help="override eps (the pairs workload also sets its pair length to eps)")
    ap.add_argument("--batch-size", type=int, default=64)
    ap.add_argument("--order-leaf", type=int, default=0,
                    help="0: balanced k-d batches; >= 1: batches of an order tree's groups")
    ap.add_argument("--group-max", type=int, default=512)
    ap.add_argument("--err-sample", type=int, default=10000)
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-6,
                    help="error target of the learned-vs-fixed comparison")
    ap.add_argument("--fallback", default=None,
                    help="the learned path's fallback and judge (n, theta) (default: "
                         "selector.fallback_for(tol))")
    ap.add_argument("--sweep", type=int, default=None,
                    help="1: time every candidate (n, theta) of the selector, plain and with "
                         "the separation rule, to find the best fixed settings at --tol "
                         "(default on for the 1e6 uniform workload); 0: only --tol-settings")
    ap.add_argument("--tol-settings", default="9,0.7,0;10,0.7,1",
                    help="n,theta,deg_min;... fixed settings timed when --sweep 0")
    ap.add_argument("--no-learned", dest="learned", action="store_false",
                    help="skip the learned (n, theta) legs")
    ap.add_argument("--precision-legs", default="fp64,fp32_kahan",
                    help="other accumulation modes timed at the headline setting")
    ap.add_argument("--oracle-sample", type=int, default=2000,
                    help="targets at which the CPU leg checks the headline against the oracle's "
                         "FP64 direct sum")
    ap.add_argument("--dual-settings", default=None,
                    help="cluster-cluster variant settings 'n,theta,target_leaf[,deg_min];...' "
                         "timed after the headline (default: two settings at E <= 1e-6 on the "
                         "1e6 uniform workload, none on the others)")
    ap.add_argument("--grid-sweep", type=int, default=None,
                    help="1: time the workload's (n, theta) grid for the Stokeslet and the "
                         "rotlet, FP64 and FP32 evaluation, E over all targets (default on for "
                         "the 100K workload c2)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB, the reference "
                         "for scaling HBM byte counters")
    args = ap.parse_args()
    if args.fallback:
        args.fallback = (int(args.fallback.split(",")[0]), float(args.fallback.split(",")[1]))
    if args.sweep is None:
        args.sweep = 1 if args.workload == "c3" and not args.n else 0
    if args.grid_sweep is None:
        args.grid_sweep = 1 if args.workload == "c2" else 0
    if args.dual_settings is None:
        args.dual_settings = "7,0.7,400;9,0.8,700" if args.workload == "c3" and not args.n else ""

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU only: the treecode path here is built and "
               "timed on a single MI355X (multi-GPU target sharding is designed, not built); "
               "run with --gpus 1")
        print(msg, file=sys.stderr)
        print(json.dumps({"error": msg, "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1902_02250_amd import bltc, inputs

    bltc.load()
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nbytes} bytes read and {nbytes} bytes written")
        del a, b
    cfg = dict(inputs.CONFIGS[args.workload])
    if args.n:
        cfg["n"] = args.n
    if args.degree:
        cfg["degree"] = args.degree
    if args.theta is not None:
        cfg["theta"] = args.theta
    if args.kernel:
        cfg["kernel"] = args.kernel
    if args.eps is not None:
        cfg["eps"] = args.eps
        if cfg["dist"] == "pairs":
            cfg["pair_length"] = args.eps
    kernel, eps, degree, theta = cfg["kernel"], cfg["eps"], cfg["degree"], cfg["theta"]
    n = cfg["n"]
    log(f"[bench] generating {args.workload}: n={n} {cfg['dist']} {kernel} eps={eps} "
        f"degree={degree} theta={theta} leaf={cfg['leaf']} precision={args.precision}")
    src = inputs.points(cfg["dist"], n, cfg["seed"], **inputs.shape_args(cfg))
    w = inputs.weights_for(cfg["dist"], n, cfg["seed"], **inputs.shape_args(cfg))
    wd = bltc.WDIM[kernel]
    if w.shape[0] != wd:   # a kernel other than the workload's own
        w = w[:wd] if w.shape[0] > wd else inputs.weights(n, cfg["seed"], wd)
    dev = torch.device("cuda:0")
    d_src = torch.from_numpy(src).to(dev)
    d_w = torch.from_numpy(w).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    tree = bltc.Tree(d_src, cfg["leaf"])
    t1 = time.perf_counter()
    tg = bltc.Targets(d_src, args.batch_size, args.order_leaf, args.group_max)
    t2 = time.perf_counter()
    log(f"[bench] tree: {tree.nnodes} clusters, depth {tree.depth} ({(t1 - t0) * 1e3:.0f} ms); "
        f"targets: {tg.nb} batches ({(t2 - t1) * 1e3:.0f} ms)")
    out = torch.empty((bltc.ODIM[kernel], n), dtype=torch.float64, device=dev)

    def step():
        tree.compute_weights(d_w, degree)
        bltc.evaluate_tree(tree, tg, kernel, eps, degree, theta, precision=args.precision,
                           out=out)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    npx, ndr = bltc.counts(tree, tg, degree, theta)
    inter = npx + ndr
    log(f"[bench] warmup done; {inter:.3e} kernel evaluations per step "
        f"({npx:.3e} far, {ndr:.3e} near)")

    bltc.profile_read(reset=True)
    bltc.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    bltc.profile_enable(False)
    prof = bltc.profile_read(reset=True)
    ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step; stages " +
        ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms" for k, v in prof.items()))

    # accuracy against the FP64 direct sum on a seeded target sample
    k = min(args.err_sample, n)
    idx = inputs.sample_indices(n, k, cfg["seed"] + 11)
    d_idx = torch.from_numpy(idx).to(dev)
    ref = bltc.direct(d_src, d_src, d_w, kernel, eps, idx=d_idx, precision="fp64")
    def errors(got):
        """E over every output row; for six rows also over u (the velocity
        of eq. error) and over w alone."""
        e = {"rel_l2_err": (torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item()}
        if got.shape[0] == 6:
            for key, r in (("rel_l2_err_u", slice(0, 3)), ("rel_l2_err_w", slice(3, 6))):
                e[key] = (torch.linalg.norm(got[r] - ref[r]) / torch.linalg.norm(ref[r])).item()
        return e

    errs = errors(out[:, d_idx])
    err = errs["rel_l2_err"]
    log(f"[bench] rel L2 error vs FP64 direct on {k} targets: " +
        ", ".join(f"{a} {b:.3e}" for a, b in errs.items()))

    ev_ms = prof["eval"][0] / max(prof["eval"][1], 1)
    flops = inter * FLOPS.get(kernel, 32)
    achieved = flops / (ev_ms * 1e-3) / 1e12
    pk = PEAK["fp64" if args.precision == "fp64" else "fp32"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": pk, "unit": "TFLOP/s",
            "frac": round(achieved / pk, 4),
            "traffic": profile_record(TRAFFIC_FILE, "traffic_bytes_per_launch", args, cfg),
            "kernel": f"k_p2p ({kernel}, {args.precision}, n={degree})",
            "achieved_kind": "algorithmic: kernel evaluations x flop per evaluation "
                             "(FMA = 2, rsqrt = 1) / launch time",
            "per_launch": f"{inter} kernel evaluations x {FLOPS.get(kernel, 32)} flop",
            "avg_launch_ms": round(ev_ms, 4)}
    executed = profile_record(COUNTER_FILE, "executed_fp32_flops_per_launch", args, cfg)
    if executed is not None:
        roof["executed"] = {"achieved": round(executed / (ev_ms * 1e-3) / 1e12, 3),
                            "frac": round(executed / (ev_ms * 1e-3) / 1e12 / pk, 4),
                            "unit": "TFLOP/s",
                            "kind": "counter-derived: 64 x SQ_INSTS_VALU_FLOPS_FP32 per launch "
                                    "(committed rocprofv3 summary of the same kernel source) "
                                    "/ launch time"}

    res = {
        "metric": "eval time & interactions/s at N=1e6, rel L2 err vs FP64 direct; "
                  "learned vs fixed (n,theta)",
        "value": inter / (ms * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: N={n} {cfg['dist']}, {kernel} "
                                f"eps={eps}, n={degree}, theta={theta}, N0={cfg['leaf']}, "
                                f"{args.precision}, batch {args.batch_size}"),
                   "n": n, "kernel": kernel, "eps": eps, "degree": degree, "theta": theta,
                   "leaf": cfg["leaf"], "precision": args.precision,
                   "batch_size": args.batch_size, "order_leaf": args.order_leaf,
                   "group_max": args.group_max},
        "eval_s": round(ms * 1e-3, 6),
        "interactions_per_step": inter,
        "direct_equivalent_per_s": float(n) * n / (ms * 1e-3),
        **errs, "err_sample": k,
        "stage_ms": {s: round(v[0] / max(v[1], 1), 4) for s, v in prof.items()},
        "build_ms": {"tree": round((t1 - t0) * 1e3, 1), "targets": round((t2 - t1) * 1e3, 1)},
        "roofline": roof,
        "cpu_baseline": None,
    }
    # the headline's output at the oracle's sample targets (for the CPU leg)
    osamp = inputs.sample_indices(n, min(args.oracle_sample, n), cfg["seed"] + 13)
    head_at_osamp = out[:, torch.from_numpy(osamp).to(dev)].cpu().numpy()

    def timed(xstep, reps):
        xstep()
        torch.cuda.synchronize()
        e0.record()
        for i in range(reps):
            r = xstep()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    # the headline in the other accumulation modes (same n, theta)
    legs = []
    for prec in [p for p in args.precision_legs.split(",") if p and p != args.precision]:
        def pstep(prec=prec):
            tree.compute_weights(d_w, degree)
            bltc.evaluate_tree(tree, tg, kernel, eps, degree, theta, precision=prec, out=out)
        xs = max(2, args.steps // 2)
        xms, _ = timed(pstep, xs)
        legs.append({"precision": prec, "steps": xs, "ms_per_step": round(xms, 4),
                     **errors(out[:, d_idx]), "interactions_per_s": inter / (xms * 1e-3)})
        log(f"[bench] headline in {prec}: {xms:.3f} ms/step, E={legs[-1]['rel_l2_err']:.3e}")
    res["precision_legs"] = legs

    # fixed settings at the error target: the listed ones, or the sweep of
    # the selector's whole candidate grid with and without the separation rule
    from paper_1902_02250_amd import selector
    if args.sweep:
        grid = [(c[0], c[1], dm) for dm in (0, selector.DEG_MIN) for c in selector.CANDIDATES]
    else:
        grid = []
        for item in [t for t in args.tol_settings.split(";") if t.strip()]:
            dn, th, dm = item.split(",")
            grid.append((int(dn), float(th), int(dm)))
    fixed = []
    for (dn, th, dm) in grid:
        def xstep(dn=dn, th=th, dm=dm):
            tree.compute_weights(d_w, dn)
            bltc.evaluate_tree(tree, tg, kernel, eps, dn, th, precision=args.precision,
                               out=out, deg_min=dm)
        xms, _ = timed(xstep, 1 if args.sweep else max(2, args.steps // 2))
        xerrs = errors(out[:, d_idx])
        fixed.append({"degree": dn, "theta": th, "deg_min": dm, "ms_per_step": round(xms, 4),
                      **xerrs})
    def best_of(rows, dm_set):
        ok = [r for r in rows if r["deg_min"] in dm_set and r["rel_l2_err"] <= args.tol]
        return min(ok, key=lambda r: r["ms_per_step"]) if ok else None
    best = {"plain": best_of(fixed, (0,)), "rule": best_of(fixed, tuple(
        sorted({r["deg_min"] for r in fixed if r["deg_min"] > 0})))}
    # the winners again, with more steps
    for key, row in best.items():
        if row is None:
            continue
        def bstep(row=row):
            tree.compute_weights(d_w, row["degree"])
            bltc.evaluate_tree(tree, tg, kernel, eps, row["degree"], row["theta"],
                               precision=args.precision, out=out, deg_min=row["deg_min"])
        xs = max(3, args.steps // 2)
        xms, _ = timed(bstep, xs)
        p_, d_ = bltc.counts(tree, tg, row["degree"], row["theta"], row["deg_min"])
        best[key] = dict(row, ms_per_step=round(xms, 4), steps=xs, **errors(out[:, d_idx]),
                         interactions_per_step=p_ + d_,
                         interactions_per_s=(p_ + d_) / (xms * 1e-3))
        log(f"[bench] best fixed ({key}) at E <= {args.tol:g}: n={row['degree']} "
            f"theta={row['theta']} deg_min={row['deg_min']}: {xms:.3f} ms/step, "
            f"E={best[key]['rel_l2_err']:.3e}")
    overall = [b for b in best.values() if b is not None]
    overall = min(overall, key=lambda r: r["ms_per_step"]) if overall else None
    # the learned (n, theta): per batch and one per run, with the fallback's
    # weights, the judge and any repair inside the timed step
    learned = []
    if not args.fallback:
        args.fallback = selector.fallback_for(args.tol)
    if args.learned and kernel in ("stokeslet", "rotlet"):
        sel = bltc.Selector(selector.MODEL_PATH)
        for mode in ("batch", "run"):
            def lstep(mode=mode):
                tree.compute_weights(d_w, args.fallback[0])
                return bltc.evaluate_adaptive(tree, tg, kernel, eps, sel, args.tol,
                                              args.fallback[0], args.fallback[1],
                                              precision=args.precision, out=out, mode=mode)
            xs = max(3, args.steps // 2)
            xms, (_, choice, stats, judge) = timed(lstep, xs)
            used = np.bincount(choice[choice >= 0], minlength=selector.K)
            row = {"mode": mode, "steps": xs, "ms_per_step": round(xms, 4),
                   **errors(out[:, d_idx]),
                   "judge_estimate": [float(judge[0]), float(judge[1])],
                   "batches_repaired": int(stats[2]), "degrees": int(stats[1]),
                   "top_choices": [[list(selector.CANDIDATES[j]), int(used[j])]
                                   for j in np.argsort(-used)[:4] if used[j]]}
            for key, b in (("best_fixed", overall), ("best_fixed_plain", best["plain"]),
                           ("best_fixed_rule", best["rule"])):
                if b is not None:
                    row[f"speedup_vs_{key}"] = round(b["ms_per_step"] / xms, 4)
            learned.append(row)
            log(f"[bench] learned ({mode}) at tol {args.tol:g}: {xms:.3f} ms/step, "
                f"E={row['rel_l2_err']:.3e}, judge {judge[0]:.2e} -> {judge[1]:.2e}, "
                f"{int(stats[2])} batches repaired, top {row['top_choices'][:2]}")
    res["learned_vs_fixed"] = {
        "tol": args.tol, "fallback": list(args.fallback),
        "grid": "selector candidates, plain and with the separation rule" if args.sweep
                else "listed settings",
        "best_fixed": overall, "best_fixed_plain": best["plain"], "best_fixed_rule": best["rule"],
        "learned": learned,
        "fixed": fixed}
    # the cluster-cluster variant on the same workload (targets = sources)
    dual = []
    for item in [t for t in args.dual_settings.split(";") if t.strip()]:
        f = item.split(",")
        dn, th, lt = int(f[0]), float(f[1]), int(f[2])
        dm = int(f[3]) if len(f) > 3 else 0
        ttree = bltc.Tree(d_src, lt)

        def dstep(dn=dn, th=th, dm=dm):
            tree.compute_weights(d_w, dn)
            return bltc.evaluate_dual(tree, ttree, kernel, eps, dn, th, precision=args.precision,
                                      out=out, deg_min=dm)[1]
        cnt = dstep()
        torch.cuda.synchronize()
        xs = max(2, args.steps // 2)
        bltc.profile_read(reset=True)
        bltc.profile_enable(True)
        e0.record()
        for i in range(xs):
            dstep()
        e1.record()
        torch.cuda.synchronize()
        bltc.profile_enable(False)
        dprof = bltc.profile_read(reset=True)
        xms = e0.elapsed_time(e1) / xs
        xerrs = errors(out[:, d_idx])
        dual.append({"degree": dn, "theta": th, "target_leaf": lt, "deg_min": dm, "steps": xs,
                     "ms_per_step": round(xms, 4), **xerrs,
                     "evaluations": {"cc": int(cnt[0]), "pc": int(cnt[1]), "cp": int(cnt[2]),
                                     "pp": int(cnt[3]), "downward": int(cnt[4])},
                     "stage_ms": {s: round(v[0] / max(v[1], 1), 4) for s, v in dprof.items()}})
        log(f"[bench] dual n={dn} theta={th} target leaf={lt} deg_min={dm}: {xms:.3f} ms/step, "
            f"E={xerrs['rel_l2_err']:.3e}, evaluations {cnt.tolist()}")
    res["dual"] = dual
    # the (n, theta) grid of the 100K workload, both kernels, FP64 against
    # FP32 evaluation with FP64 sums, E over every target
    if args.grid_sweep:
        gs = []
        for gk in ("stokeslet", "rotlet"):
            gref = bltc.direct(d_src, d_src, d_w, gk, eps, precision="fp64")
            gout = torch.empty((bltc.ODIM[gk], n), dtype=torch.float64, device=dev)
            for dn in cfg.get("degrees", (2, 4, 6, 8, 10)):
                for th in cfg.get("thetas", (0.5, 0.7, 0.9)):
                    row = {"kernel": gk, "degree": dn, "theta": th}
                    for prec in ("fp64", "fp32_fp64acc"):
                        def gstep(dn=dn, th=th, prec=prec, gk=gk):
                            tree.compute_weights(d_w, dn)
                            bltc.evaluate_tree(tree, tg, gk, eps, dn, th, precision=prec,
                                               out=gout)
                        gms, _ = timed(gstep, 3)
                        gE = (torch.linalg.norm(gout - gref) / torch.linalg.norm(gref)).item()
                        row[prec] = {"ms_per_step": round(gms, 4), "rel_l2_err": gE}
                    p_, d_ = bltc.counts(tree, tg, dn, th)
                    row["interactions_per_step"] = p_ + d_
                    gs.append(row)
                    log(f"[bench] grid {gk} n={dn} theta={th}: FP64 "
                        f"{row['fp64']['ms_per_step']:.2f} ms E={row['fp64']['rel_l2_err']:.2e}; "
                        f"FP32 {row['fp32_fp64acc']['ms_per_step']:.2f} ms "
                        f"E={row['fp32_fp64acc']['rel_l2_err']:.2e}")
        res["grid_sweep"] = {"targets": n, "err": "all targets against the FP64 direct sum",
                             "rows": gs}
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline on {args.cpu_sample} targets ...")
        res["cpu_baseline"] = cpu_baseline(cfg, src, w, args.cpu_sample, args, osamp,
                                           head_at_osamp)
        res["rel_l2_err_oracle"] = res["cpu_baseline"]["rel_l2_err_oracle"]
        res["err_sample_oracle"] = int(osamp.size)
        log(f"[bench] CPU oracle: {res['cpu_baseline']['value']:.3e} interactions/s "
            f"({res['cpu_baseline']['seconds']:.1f} s); headline E vs the oracle's direct sum "
            f"on {osamp.size} targets {res['rel_l2_err_oracle']:.3e}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
