"""Benchmark: exact all-kNN queries/s on one MI355X.

One step = the whole job on inputs already resident in HBM: build the
reference kd-tree, build the query kd-tree, run the pruning dual-tree search,
write the (index, distance) lists.  The plain path is one knn_all_knn call
(builds overlapped on two streams, search, one stream synchronisation); with
the learned seed the trees are built first, the seed network runs on them,
then the search.  W untimed warm-up steps, then K timed steps between device
synchronisations.  Prints ONE JSON line.

Headline workload: 1,000,000 reference x 1,000,000 query points, d = 3,
32-component Gaussian mixture, k = 10, leaf size 32, FP32 path.

The second half of the metric -- learned seed + BF16 tiles against the plain
FP32 traversal -- is measured on the workload where the combined variant is
defined (1,000,000 reference x 262,144 query points on a 10-dim manifold in
d = 64, k = 50) and reported in the "compare" object, with the plain BF16
variant and the classic B1 bound beside it.  Every timed variant's answer is
checked against the FP64 oracle on the seeded sample that the CPU baseline
times.

The dominant kernel is the traversal kernel; its average duration comes
from HIP events the library records around that launch on the same stream
(knn_stats.ms_main_kernel).  Algorithmic FLOPs per evaluated pair are
3d - 1 (direct difference: d subtractions, d squares, d - 1 additions).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "fp32_vector_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "bf16_mfma_tflops": 2500.0,
    "hbm_gbs": 8000.0,
}

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
# counter reads for a plain 1 GiB device copy (--copy-calibration): FETCH_SIZE
# x 2.000, WRITE_SIZE x 1.000.  Only workloads whose kernel is unchanged since
# the counters were taken appear here.
TRAFFIC_BYTES_PER_LAUNCH = {
    ("gmm1m_d3_k10", "fp32"): int((342779.5 * 2.000 + 158830.5625 * 1.000) * 1024),
    ("manifold1m_d64_k50", "bf16"): int((182753836.3125 * 2.000 + 265397.375 * 1.000) * 1024),
}

COMBINED_WORKLOAD = "manifold1m_d64_k50"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gmm1m_d3_k10")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--bound", default="B", choices=["B", "B1", "none"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned", action="store_true",
                    help="train the seed network on 8 other seeded draws of the workload "
                         "(untimed), then time steps that include seed inference")
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--target-fallback", type=float, default=0.005,
                    help="seed calibration: share of held-out leaves allowed above the seed")
    ap.add_argument("--compare", action="store_true",
                    help="also time the plain FP32 path on the same workload and report "
                         "the speedup of the chosen variant over it")
    ap.add_argument("--no-combined", action="store_true",
                    help="skip the learned+BF16 vs plain FP32 comparison on the d = 64 workload")
    ap.add_argument("--combined-train-seeds", type=int, default=4)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the k-furthest, range, KDE and EMST measurements")
    ap.add_argument("--only-extras", action="store_true",
                    help="run only the k-furthest, range, KDE and EMST measurements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (reference "
                         "kernel for scaling the HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4,
                                           "launches": 3}}))


def cpu_baseline(ref, q, k, self_mode, target_s, answers=None):
    """The oracle (FP64 brute force, OpenMP, all host cores) timed on a
    seeded sample of the same queries, scaled to queries/s.  The same
    sample then checks each GPU answer in ``answers`` ({name: (idx, dist)},
    host arrays) with the acceptance predicate."""
    import numpy as np

    from oracle import knn as ok
    from oracle import parity
    qq = ref if self_mode else q
    rng = np.random.default_rng(1234)
    n = 64
    elapsed = 0.0
    while True:
        rows = np.sort(rng.choice(len(qq), size=min(n, len(qq)), replace=False))
        t0 = time.perf_counter()
        oi, od = ok.knn_rows(qq, rows, ref, k, exclude_self=self_mode)
        elapsed = time.perf_counter() - t0
        if elapsed >= 0.8 * target_s or n >= len(qq):
            break
        # next sample sized for the target (growth capped, so a slow first
        # estimate cannot overshoot far)
        n = int(min(len(qq), n * min(16.0, max(1.5, target_s / max(elapsed, 1e-3) * 1.05))))
    out = {"value": len(rows) / elapsed, "unit": "queries/s", "cores": ok.threads(),
           "kind": "oracle",
           "sample": f"{len(rows)} seeded queries x all {len(ref)} references "
                     f"(FP64 brute force), {elapsed:.2f} s"}
    if answers:
        out["parity"] = {}
        for name, (gi, gd) in answers.items():
            fails, info = parity.check(qq, ref, k, gi, gd, oi, od, rows=rows,
                                       exclude_self=self_mode)
            out["parity"][name] = {"rows": info["rows"], "ok": not any(fails.values()),
                                   "identical_sets": info["identical_sets"],
                                   "failures": {a: b for a, b in fails.items() if b}}
    return out


def _timed(run, steps, warmup):
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sts.append(run())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, sts


def seed_ceiling(R, Q, k, leaf, precision, reps=3):
    """What any learned seed could gain at best: the seeded search with the
    ideal seed -- each query leaf's true largest k-th distance, reported by
    a plain run (leaf_kth_out), nudged up so that no leaf falls back --
    against the plain search, both on the same prebuilt trees."""
    import numpy as np
    import torch

    from paper_1304_4327_amd import knn
    rt, qt = knn.knn_build_tree_pair(R, Q, leaf)
    nl = qt.info()["n_leaves"]
    kth = torch.empty(nl, dtype=torch.float32, device="cuda")
    knn.knn_search(rt, qt, k, precision=precision, leaf_kth_out=kth)
    ideal = (kth.double() * (1 + 1e-5)).float().contiguous()

    def run(seed):
        return knn.knn_search(rt, qt, k, precision=precision, seed_radius=seed, stats=True)[2]

    out = {}
    for name, seed in (("plain", None), ("ideal_seed", ideal)):
        run(seed)
        sts = [run(seed) for _ in range(reps)]
        out[name] = {"ms_search": float(np.mean([s["ms_search"] for s in sts])),
                     "pairs_per_query": sts[0]["pairs"] / Q.shape[0],
                     "fallback_leaves": sts[0]["fallback_leaves"]}
    out["speedup_of_ideal_seed"] = out["plain"]["ms_search"] / out["ideal_seed"]["ms_search"]
    qt.close()
    rt.close()
    return out


def combined(args):
    """Learned seed + BF16 tiles against the plain FP32 traversal on the d = 64
    workload (plus plain BF16, and the B1 bound), every variant checked."""
    import numpy as np
    import torch

    from paper_1304_4327_amd import datagen, knn
    from paper_1304_4327_amd import seed as S
    name = COMBINED_WORKLOAD
    ref, q, k, leaf = datagen.make(name)
    R, Q = torch.from_numpy(ref).cuda(), torch.from_numpy(q).cuda()
    nq = len(q)
    base = datagen.DEFAULT_SEEDS[name]
    seeds = [base + 100 + i for i in range(args.combined_train_seeds)]
    t0 = time.perf_counter()
    model = S.train_for_workload(name, seeds, epochs=args.train_epochs, precision="bf16",
                                 target_fallback=args.target_fallback)
    train_s = time.perf_counter() - t0
    print(f"combined: seed network trained in {train_s:.1f} s", file=sys.stderr, flush=True)

    def plain(precision, bound="B"):
        return lambda: knn.knn_all_knn(R, Q, k, leaf, bound=bound, precision=precision,
                                       stats=True)

    def learned():
        rt, qt = knn.knn_build_tree_pair(R, Q, leaf)
        rad = S.radii(model, knn.knn_seed_features(rt, qt))
        out = knn.knn_search(rt, qt, k, precision="bf16", seed_radius=rad, stats=True)
        qt.close()
        rt.close()
        return out

    res, answers = {}, {}
    for key, run, steps, warm in (("plain_fp32", plain("fp32"), 2, 1),
                                  ("learned_bf16", learned, 4, 1),
                                  ("plain_bf16", plain("bf16"), 4, 1),
                                  ("plain_bf16_B1", plain("bf16", "B1"), 2, 1)):
        ms, outs = _timed(run, steps, warm)
        sts = [o[2] for o in outs]
        res[key] = {"ms_per_step": ms, "queries_per_s": nq / ms * 1e3,
                    "pairs_per_query": float(np.mean([s["pairs"] for s in sts])) / nq,
                    "score_calls_per_query": float(np.mean([s["score_calls"] for s in sts])) / nq,
                    "ms_search": float(np.mean([s["ms_search"] for s in sts]))}
        if key == "learned_bf16":
            res[key]["fallback_leaves"] = float(np.mean([s["fallback_leaves"] for s in sts]))
            res[key]["query_leaves"] = sts[0]["n_query_leaves"]
        answers[key] = (outs[-1][0].cpu().numpy(), outs[-1][1].cpu().numpy())
        print(f"combined: {key} {ms:.2f} ms/step", file=sys.stderr, flush=True)
    ceiling = seed_ceiling(R, Q, k, leaf, "bf16")
    print(f"combined: ideal seed {ceiling['speedup_of_ideal_seed']:.3f}x", file=sys.stderr,
          flush=True)
    line = {"workload": name, "n_ref": len(ref), "n_query": nq, "d": ref.shape[1], "k": k,
            "baseline": "plain FP32 dual-tree traversal, bound B",
            "speedup_learned_bf16_vs_plain_fp32":
                res["plain_fp32"]["ms_per_step"] / res["learned_bf16"]["ms_per_step"],
            "speedup_plain_bf16_vs_plain_fp32":
                res["plain_fp32"]["ms_per_step"] / res["plain_bf16"]["ms_per_step"],
            "bound_B_vs_B1_pairs_per_query": [res["plain_bf16"]["pairs_per_query"],
                                              res["plain_bf16_B1"]["pairs_per_query"]],
            "variants": res,
            "seed_training": {"train_seeds": seeds, "eval_seed": base, "train_s": train_s,
                              "log_margin": model.log_margin},
            "seed_ceiling_bf16": ceiling}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ref, q, k, False, 5.0, answers)
    return line


def extras(args):
    """The other instances of the meta-algorithm, each timed on the d = 3
    Gaussian-mixture workload (1M references, 1M queries, leaf 32) with
    prebuilt trees, its dominant kernel's roofline figure, and the oracle
    timed on a sample that also checks the answer."""
    import numpy as np
    import torch

    from paper_1304_4327_amd import datagen, knn
    ref, q, k, leaf = datagen.make("gmm1m_d3_k10")
    d = ref.shape[1]
    R, Q = torch.from_numpy(ref).cuda(), torch.from_numpy(q).cuda()
    rt, qt = knn.knn_build_tree_pair(R, Q, leaf)
    peak = PEAKS["fp32_vector_tflops"]
    out = {"workload": "gmm1m_d3_k10", "n_ref": len(ref), "n_query": len(q), "d": d,
           "leaf_size": leaf, "timed": "the operation on prebuilt trees (device events)"}

    def roof(pairs, flop, ms):
        ach = pairs * flop / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "flop_per_pair": flop, "pairs_per_launch": pairs}

    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(len(q), 1024, replace=False))

    # k-furthest neighbours, k = 10
    ms, outs = _timed(lambda: knn.knn_search_furthest(rt, qt, k, stats=True), 3, 1)
    st = outs[-1][2]
    far = {"k": k, "ms": st["ms_search"], "queries_per_s": len(q) / st["ms_search"] * 1e3,
           "pairs_per_query": st["pairs"] / len(q),
           "roofline": roof(st["pairs"], 3 * d - 1, st["ms_search"])}
    gi, gd = outs[-1][0].cpu().numpy(), outs[-1][1].cpu().numpy()
    print(f"extras: furthest {st['ms_search']:.2f} ms", file=sys.stderr, flush=True)
    # range search, [0, 0.2]
    lo, hi = 0.0, 0.2
    ms, outs = _timed(lambda: knn.knn_range_search(rt, qt, lo, hi, stats=True), 3, 1)
    sc, sf = outs[-1][3]
    off = outs[-1][0].cpu().numpy()
    rng_ = {"lo": lo, "hi": hi, "ms_count": sc["ms_search"], "ms_fill": sf["ms_search"],
            "neighbours_per_query": float(off[-1]) / len(q),
            "queries_per_s": len(q) / (sc["ms_search"] + sf["ms_search"]) * 1e3,
            "pairs_per_query": sc["pairs"] / len(q),
            "roofline": roof(sc["pairs"], 3 * d - 1, sc["ms_search"])}
    rng_ans = (off, outs[-1][1].cpu().numpy())
    print(f"extras: range {sc['ms_search']:.2f} + {sf['ms_search']:.2f} ms", file=sys.stderr,
          flush=True)
    # kernel density sums, h = 1, eps = 1
    h, eps = 1.0, 1.0
    ms, outs = _timed(lambda: knn.knn_kde(rt, qt, h, eps, stats=True), 3, 1)
    st = outs[-1][1]
    kde = {"h": h, "eps": eps, "ms": st["ms_search"],
           "queries_per_s": len(q) / st["ms_search"] * 1e3,
           "pairs_per_query": st["pairs"] / len(q),
           "approximated_nodes_per_query": st["inserts"] / len(q),
           # distance (3d - 1), scaling and exponential counted one each
           "roofline": roof(st["pairs"], 3 * d + 1, st["ms_search"])}
    f = outs[-1][0].cpu().numpy()
    print(f"extras: kde {st['ms_search']:.2f} ms", file=sys.stderr, flush=True)
    # minimum spanning tree of the reference set
    ms, outs = _timed(lambda: knn.knn_emst(rt, stats=True), 2, 1)
    u, v, w, rounds, st = outs[-1]
    emst = {"n": len(ref), "ms": st["ms_search"], "rounds": rounds,
            "points_per_s": len(ref) / st["ms_search"] * 1e3,
            "pairs_per_point": st["pairs"] / len(ref),
            "total_length": float(w.double().sum().item()),
            "roofline": roof(st["pairs"], 3 * d - 1, st["ms_search"])}
    print(f"extras: emst {st['ms_search']:.2f} ms, {rounds} rounds", file=sys.stderr, flush=True)
    qt.close()
    rt.close()
    if not args.no_cpu_baseline:
        base = extras_cpu_baseline(ref, q, k, rows, (gi, gd), rng_ans, (lo, hi), f, (h, eps),
                                   (u.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy()))
        far["cpu_baseline"], rng_["cpu_baseline"], kde["cpu_baseline"], emst["cpu_baseline"] = base
    out.update(k_furthest=far, range_search=rng_, kde=kde, emst=emst)
    return out


def extras_cpu_baseline(ref, q, k, rows, far_ans, rng_ans, rng_lohi, kde_f, kde_he, emst_uvw):
    """The oracle for each extra timed on a seeded sample, which also checks
    the GPU answer on that sample (range: identical sets; furthest: the
    acceptance predicate; KDE: within eps plus the FP32 budget; EMST: the
    total length of the 1M tree against no oracle -- Prim's O(n^2) is timed
    on a 20k-point prefix and its tree checked against the GPU's on that
    prefix)."""
    import numpy as np
    import torch

    from oracle import knn as ok
    from oracle import parity
    from paper_1304_4327_amd import knn
    cores = ok.threads()
    res = []
    t0 = time.perf_counter()
    oi, od = ok.furthest_rows(q, rows, ref, k)
    el = time.perf_counter() - t0
    fails, _ = parity.check_furthest(q, ref, k, far_ans[0], far_ans[1], oi, od, rows=rows)
    res.append({"value": len(rows) / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
                "sample": f"{len(rows)} seeded queries, {el:.2f} s",
                "parity_ok": not any(fails.values())})
    lo, hi = rng_lohi
    t0 = time.perf_counter()
    oo, oidx, _ = ok.range_rows(q, rows, ref, lo, hi)
    el = time.perf_counter() - t0
    off, idx = rng_ans
    same = all(np.array_equal(np.sort(idx[off[r]:off[r + 1]]), oidx[oo[t]:oo[t + 1]])
               for t, r in enumerate(rows))
    res.append({"value": len(rows) / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
                "sample": f"{len(rows)} seeded queries, {el:.2f} s", "parity_ok": bool(same)})
    h, eps = kde_he
    t0 = time.perf_counter()
    fe, budget = ok.kde_rows(q, rows, ref, h)
    el = time.perf_counter() - t0
    good = bool(np.all(np.abs(kde_f[rows] - fe) <= eps * (1 + 1e-5) + 2e-5 * budget))
    res.append({"value": len(rows) / el, "unit": "queries/s", "cores": cores, "kind": "oracle",
                "sample": f"{len(rows)} seeded queries, {el:.2f} s", "parity_ok": good})
    sub = ref[:20000]
    t0 = time.perf_counter()
    pu, pv, _ = ok.emst(sub)
    el = time.perf_counter() - t0
    tr = knn.knn_build_tree(torch.from_numpy(sub).cuda(), 32)
    gu, gv, _, _, _ = knn.knn_emst(tr)
    same = np.array_equal(ok.edge_set(pu, pv), ok.edge_set(gu.cpu().numpy(), gv.cpu().numpy()))
    tr.close()
    res.append({"value": len(sub) / el, "unit": "points/s (Prim, O(n^2))", "cores": cores,
                "kind": "oracle", "sample": f"the first 20000 reference points, {el:.2f} s",
                "parity_ok": bool(same)})
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark use one GPU only; "
                                   "--gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.only_extras:
        print(json.dumps({"extras": extras(args)}), flush=True)
        return
    import numpy as np
    import torch

    from paper_1304_4327_amd import datagen, knn

    ref, q, k, leaf = datagen.make(args.workload)
    self_mode = q is None
    d = ref.shape[1]
    R = torch.from_numpy(ref).cuda()
    Q = None if self_mode else torch.from_numpy(q).cuda()
    nq = len(ref) if self_mode else len(q)
    idx = torch.empty((nq, k), dtype=torch.int64, device="cuda")
    dist = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    model = None
    train_info = None
    if args.learned:
        from paper_1304_4327_amd import seed as S
        base = datagen.DEFAULT_SEEDS[args.workload]
        train_seeds = list(range(40, 48)) if args.workload == "zipfgmm2m_d8_k10" else \
            [base + 100 + i for i in range(8)]
        t0 = time.perf_counter()
        model = S.train_for_workload(args.workload, train_seeds, epochs=args.train_epochs,
                                     precision=args.precision,
                                     target_fallback=args.target_fallback)
        train_info = {"train_seeds": train_seeds, "eval_seed": base,
                      "target_fallback": args.target_fallback,
                      "train_s": time.perf_counter() - t0, "log_margin": model.log_margin,
                      "loss_first": model.history[0], "loss_last": model.history[-1]}

    def step(precision, learned=False):
        if not learned:
            # the whole path in one library call: both builds (overlapped on
            # two streams), the search, one stream synchronisation
            _, _, st = knn.knn_all_knn(R, None if self_mode else Q, k, leaf, bound=args.bound,
                                       precision=precision, exclude_self=self_mode, stats=True,
                                       out=(idx, dist), stream=stream)
            return st
        # learned seed: the seed features need the trees between build and search
        if self_mode:
            rt, qt = knn.knn_build_tree(R, leaf, stream=stream), None
        else:
            rt, qt = knn.knn_build_tree_pair(R, Q, leaf, stream=stream)
        from paper_1304_4327_amd import seed as S
        rad = S.radii(model, knn.knn_seed_features(rt, qt, stream=stream))
        _, _, st = knn.knn_search(rt, qt, k, bound=args.bound, precision=precision,
                                  exclude_self=self_mode, stats=True, out=(idx, dist),
                                  seed_radius=rad, stream=stream)
        st["ms_ref_build"] = rt.info()["ms_build"]
        if qt is not None:
            st["ms_query_build"] = qt.info()["ms_build"]
            qt.close()
        rt.close()
        return st

    def timed(precision, steps, warmup, learned=False):
        for _ in range(warmup):
            step(precision, learned)
        torch.cuda.synchronize()
        sts = []
        t0 = time.perf_counter()
        for _ in range(steps):
            sts.append(step(precision, learned))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sts

    total, stats = timed(args.precision, args.steps, args.warmup, args.learned)
    ms_step = total / args.steps * 1e3
    value = nq * args.steps / total
    answer = (idx.cpu().numpy(), dist.cpu().numpy())
    compare = None
    if args.compare:
        base_total, base_stats = timed("fp32", max(1, min(args.steps, 2)), 1)
        base_ms = base_total / max(1, min(args.steps, 2)) * 1e3
        compare = {"baseline": "plain FP32 dual-tree (same workload, same bound)",
                   "baseline_ms_per_step": base_ms, "variant_ms_per_step": ms_step,
                   "speedup": base_ms / ms_step,
                   "baseline_pairs_per_query": float(np.mean([s["pairs"] for s in base_stats])) / nq}

    kern_ms = float(np.mean([s["ms_main_kernel"] for s in stats]))
    pairs = float(np.mean([s["pairs"] for s in stats]))
    if args.precision == "bf16":
        # BF16 MFMA: 2 d flops per pair on the matrix cores (padded k-steps
        # of 16 count as issued work, the algorithmic count uses d)
        flop_per_pair = 2 * d
        peak = PEAKS["bf16_mfma_tflops"]
        # the BF16 kernel the library picks: the leaf sweep at stride 64,
        # the traversal kernel with matrix-core tiles at stride 16 / 32 with
        # lists of <= 16, else the per-leaf MFMA kernel
        stride = 16 if d <= 16 else 32 if d <= 32 else 64
        bound_kind = "mfma"
        kname = ("k_search_mfma_sweep" if stride == 64 else
                 "k_search_valu_mt" if k + (1 if self_mode else 0) <= 16 else "k_search_mfma")
    else:
        flop_per_pair = 3 * d - 1
        peak = PEAKS["fp32_vector_tflops"]
        bound_kind, kname = "alu", "k_search_valu"
    achieved = pairs * flop_per_pair / (kern_ms * 1e-3) / 1e12
    traffic = None if args.learned else TRAFFIC_BYTES_PER_LAUNCH.get((args.workload, args.precision))
    line = {
        "metric": "exact kNN queries/s, 1M×1M d=3 k=10; learned+BF16 vs plain FP32 speedup",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64" if args.precision == "bf16" else "f32",
        "data": "synthetic (seeded, generated on the host; no dataset)",
        "config": {"workload": args.workload, "n_ref": len(ref), "n_query": nq, "d": d, "k": k,
                   "leaf_size": leaf, "bound": args.bound, "precision": args.precision,
                   "learned_seed": bool(args.learned), "parallelism": "single GPU"},
        "roofline": {"bound": bound_kind, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": kname, "kernel_ms": kern_ms,
                     "flop_per_pair": flop_per_pair, "pairs_per_launch": pairs},
        "breakdown_ms": {
            "ref_build": float(np.mean([s["ms_ref_build"] for s in stats])),
            "query_build": float(np.mean([s.get("ms_query_build", 0.0) for s in stats])),
            "search": float(np.mean([s["ms_search"] for s in stats])),
        },
        "pairs_per_query": pairs / nq,
        "score_calls": float(np.mean([s["score_calls"] for s in stats])),
    }
    if compare:
        line["compare"] = compare
    if args.learned:
        line["learned"] = dict(train_info,
                               fallback_leaves=float(np.mean([s["fallback_leaves"] for s in stats])),
                               fallback_queries=float(np.mean([s["fallback_queries"] for s in stats])),
                               query_leaves=stats[0]["n_query_leaves"],
                               fallback_query_rate=float(np.mean([s["fallback_queries"] for s in stats])) / nq,
                               fallback_pairs_per_query=float(np.mean([s["fallback_pairs"] for s in stats])) / nq,
                               ms_seeded_pass=float(np.mean([s["ms_main_kernel"] for s in stats])),
                               ms_search_total=float(np.mean([s["ms_search"] for s in stats])))
    if not self_mode and not args.learned:
        line["seed_ceiling"] = seed_ceiling(R, Q, k, leaf, args.precision)
    if d == 3 and args.precision == "fp32" and not args.learned and args.bound == "B":
        # the BaseCase tiles alone: the search's recorded leaf list replayed
        # without the walk (same tiles, same order, same answer)
        rt, qt = (knn.knn_build_tree(R, leaf), None) if self_mode else \
            knn.knn_build_tree_pair(R, Q, leaf)
        reps = [knn.knn_debug_tile_replay(rt, qt, k, exclude_self=self_mode) for _ in range(3)]
        tile_ms = float(np.mean([r[3] for r in reps]))
        tile_pairs = reps[-1][4]
        tach = tile_pairs * flop_per_pair / (tile_ms * 1e-3) / 1e12
        line["roofline"].update(tile_ms=tile_ms, tile_achieved=tach, tile_frac=tach / peak,
                                tile_note="the search's BaseCase tiles (distances, filter, "
                                          "k-list inserts, bound refresh) replayed without "
                                          "the walk and Score")
        if qt is not None:
            qt.close()
        rt.close()
    print(f"headline done: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ref, q, k, self_mode, args.cpu_seconds,
                                            {"headline": answer})
    del R, Q, idx, dist
    if not args.no_combined and args.workload != COMBINED_WORKLOAD:
        torch.cuda.empty_cache()
        line["compare_learned_bf16"] = combined(args)
    if not args.no_extras:
        torch.cuda.empty_cache()
        line["extras"] = extras(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
