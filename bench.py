#!/usr/bin/env python3
"""Benchmark of the FUnc-SNE step on one MI355X.

Workload: 1,000,000 points on 50 seeded 8-dim linear manifolds in R^128
(FP32 rows), embedded in d = 16 with K_hd = K_ld = 32, 16 negatives,
alpha = 1, perplexity 10.  A timed step is one full iteration with the HD
refinement on (every row of the step runs: coin, candidates, HD distances,
merge, recalibration, affinities, LD refinement, gradient, Z, update).

Prints one JSON line.  Besides the headline it reports the per-kernel
roofline of the dominant kernel (of those with algorithmic bytes, the one
that takes longest per step), the other kernels, the
1000-iteration run of the workload under the refinement coin for the FP32
and the BF16 forms (wall seconds and HD recall@32 on a query sample), and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "embedding iters/s at N=1M (HD KNN recall@K, HBM GB/s); BF16/MLP vs FP32"
PEAK_HBM_GBS = 8000.0
C_SLOTS = 32


# Sources the step's kernels and their launches are built from; the placement
# network, clustering and jump-start files hold kernels of their own.
STEP_SOURCES = ("fsne_api.hip", "fsne_bf16.hip", "fsne_unit.hip", "fsne_reorder.hip",
                "fsne_context.h", "fsne_device.h",
                "fsne_kernels.h", "fsne_kernels.hip")


def kernel_source_hash() -> str:
    """Hash of the step kernels' sources: counter readings taken with other
    sources are not reported."""
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_07681_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def memo_width(D, xbytes, dist_mode=0):
    """Remembered HD rejections per point (each read, then rewritten)."""
    return 64 if dist_mode == 0 and D * xbytes >= 512 else 32


def bytes_per_point(cfg, xbytes, hd_cand, ld_cand):
    """Bytes each kernel must move per point, no cache reuse assumed.

    hd_cand / ld_cand: mean number of distinct candidate rows per point that
    the kernels loaded (duplicate slots and remembered rejections are dropped
    before any row is read).
    """
    D, d, Kh, Kl, nn = cfg["D"], cfg["d"], cfg["K_hd"], cfg["K_ld"], cfg["n_neg"]
    dp = 2
    while dp < d:
        dp *= 2
    sx, sy = D * xbytes, 4 * dp
    hd = sx * (1 + hd_cand) + 16 * Kh + 4 * Kl + 96 + 33 + 8 * memo_width(D, xbytes)
    ld = sy * (1 + Kl + ld_cand + Kh + nn + 2) + 8 * Kh + 8 * Kl + 96 + 5
    upd = 6 * sy
    return dict(hd_refine=hd, ld_grad=ld, update=upd)


def all_slot_bytes_per_point(cfg, xbytes):
    """The same with every one of the 32 candidate slots counted."""
    D, d, Kh, Kl, nn = cfg["D"], cfg["d"], cfg["K_hd"], cfg["K_ld"], cfg["n_neg"]
    sx, sy = D * xbytes, 4 * d
    hd = (C_SLOTS + 1) * sx + 96 + 16 * Kh + 12 + 24 * Kh + 12 + 8 * memo_width(D, xbytes)
    ld = sy + 8 * Kl + 8 * Kh + 96 + (Kl + C_SLOTS + Kh + nn) * sy + 2 * sy
    return dict(hd_refine=hd, ld_grad=ld, update=6 * sy)


def progress(msg):
    """A line on stderr as each leg ends (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def reorder_due(t, every, start):
    """Whether the points are renumbered before iteration t: every `every`
    iterations from iteration `start` on (before it the embedding has no
    structure that a renumbering could follow)."""
    return every > 0 and t >= start and (t - start) % every == 0


def track_renumbering(orig, p):
    """orig[k] = original id of current point k; point k becomes p[k]."""
    if orig is not None:
        nxt = orig.copy()
        nxt[p] = orig
        orig[:] = nxt


def run_steps(emb, t0, n, every, start, orig=None):
    """Iterations t0 .. t0+n-1, the points renumbered along the Morton order of
    the embedding (fsne_reorder) where reorder_due says so (orig, if given,
    follows the original id of each point)."""
    t = t0
    while t < t0 + n:
        if reorder_due(t, every, start):
            track_renumbering(orig, emb.reorder())
        nxt = t + 1
        while nxt < t0 + n and not reorder_due(nxt, every, start):
            nxt += 1
        emb.step(nxt - t)
        t = nxt


def profiled_steps(emb, t0, n, every, start, N, orig=None):
    """Iterations t0 .. t0+n-1 one at a time with kernel timing on (HIP events
    on the library's stream), renumbering as run_steps; returns the kernel
    times and the mean HD / LD candidate rows per point."""
    import numpy as np

    emb.profile(True)
    hd_c, ld_c = [], []
    for t in range(t0, t0 + n):
        if reorder_due(t, every, start):
            track_renumbering(orig, emb.reorder())
        emb.step(1)
        s1 = emb.stats()
        hd_c.append(s1["hd_cand_rows"] / N)
        ld_c.append(s1["ld_cand_rows"] / N)
    kt = emb.kernel_times()
    emb.profile(False)
    return kt, float(np.mean(hd_c)), float(np.mean(ld_c))


def schedule(F, base, t):
    """Early exaggeration 12 with momentum 0.5 for 250 iterations, then 1 and 0.8."""
    early = t < 250
    return F.fsne_default_hparams(**{**base, "attr": 12.0 if early else 1.0,
                                     "momentum": 0.5 if early else 0.8})


def quality_run(F, X, cfg, Y0, n_iter, seed, queries, ex_d2, dist_mode=0, every=50,
                labels=None, lr_div=12.0, reorder_every=0, reorder_data=False):
    """n_iter iterations under the coin with the standard schedule; HD recall@K
    on the query sample every ``every`` iterations (the clock is stopped while
    the recall is measured).  With reorder_every > 0 the points are renumbered
    along the embedding's Morton order at every multiple of it (timed), with
    reorder_data along a projection of the data rows before the first
    iteration (timed); the lists are mapped back to the original ids to be
    measured."""
    import numpy as np

    from inputs.knn_metrics import recall_at_k

    N = X.shape[0]
    base = dict(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N / lr_div,
                n_neg=cfg["n_neg"], hd_mode=0, dist_mode=dist_mode)
    emb = F.Embedding(X, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=seed,
                      hp=schedule(F, base, 0))
    emb.sync()
    r0 = emb.stats()["hd_refinements"]
    orig = np.arange(N)              # original id of each current id

    def in_original_ids(lists):
        out = np.empty_like(lists)
        out[orig] = orig[lists]
        return out

    done, secs, curve = 0, 0.0, []
    if reorder_data:
        t0 = time.perf_counter()
        track_renumbering(orig, emb.reorder_data())
        emb.sync()
        secs += time.perf_counter() - t0
    while done < n_iter:
        stop = min(n_iter, (done // every + 1) * every)
        if done < 250 < stop:
            stop = 250
        emb.set_hyperparams(schedule(F, base, done))
        t0 = time.perf_counter()
        if reorder_every > 0 and done > 0 and done % reorder_every == 0:
            p = emb.reorder()
            nxt = np.empty_like(orig)
            nxt[p] = orig
            orig = nxt
        emb.step(stop - done)
        emb.sync()
        secs += time.perf_counter() - t0
        done = stop
        if done % every == 0 or done == n_iter:
            if done % 500 == 0:
                progress(f"run (dist_mode {dist_mode}): iteration {done}")
            idx, _ = emb.knn(0)
            curve.append([done, round(secs, 4),
                          round(recall_at_k(in_original_ids(idx), X, queries, ex_d2), 4)])
    st = emb.stats()
    extra = {}
    if labels is not None:
        ld = in_original_ids(emb.knn(1)[0])
        extra["ld_same_class"] = round(float((labels[ld] == labels[:, None]).mean()), 4)
    emb.close()
    return dict(**extra, iters=n_iter, seconds=round(secs, 3), iters_per_s=round(n_iter / secs, 2),
                hd_refinements=int(st["hd_refinements"] - r0),
                recall_at_32=curve[-1][2], final_E=round(float(st["E"]), 4),
                nonfinite=int(st["nonfinite"]), curve=curve)


def seconds_to(curve, target):
    """Step seconds at which the recall curve first reaches target, linearly
    interpolated between the two checkpoints around the crossing (None if it
    never does)."""
    prev = (0, 0.0, 0.0)
    for it, secs, rec in curve:
        if rec >= target:
            _, s0, r0 = prev
            return round(s0 + (secs - s0) * (target - r0) / (rec - r0), 4) if rec > r0 else secs
        prev = (it, secs, rec)
    return None


def cpu_baseline(X, cfg, Y0, seed, n_one=200_000):
    """The FP64 oracle on the host: one HD-refining iteration over all N points
    on every thread, and the same on one thread over the first n_one rows (a
    uniform sample: the rows are shuffled), scaled to N by the point count."""
    from oracle import oracle as O

    N = X.shape[0]
    hp = O.Hyper(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=float(N / 12.0),
                 momentum=0.5, attr=12.0, n_neg=cfg["n_neg"], hd_mode=1)
    S = O.OracleState(X, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed, Y0).init(hp)
    t0 = time.perf_counter()
    S.step(hp)
    dt = time.perf_counter() - t0
    del S
    threads = O.num_threads()
    O.set_num_threads(1)
    try:
        S1 = O.OracleState(X[:n_one], cfg["d"], cfg["K_hd"], cfg["K_ld"], seed, Y0[:n_one])
        S1.init(hp.copy(lr=float(n_one / 12.0)))
        t1 = time.perf_counter()
        S1.step(hp.copy(lr=float(n_one / 12.0)))
        dt1 = time.perf_counter() - t1
        del S1
    finally:
        O.set_num_threads(threads)
    return {"value": round(1.0 / dt, 4), "unit": "iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"1 iteration with the HD refinement on, over all N={N} points of the "
                      "same workload (FP64 C oracle, OpenMP over points), after an untimed "
                      f"oracle init; {dt:.2f} s",
            "single_thread": {"value": round(n_one / (N * dt1), 5), "unit": "iters/s",
                              "cores": 1, "kind": "oracle",
                              "sample": f"1 HD-refining iteration over the first {n_one} rows "
                                        f"(a uniform sample of the shuffled workload) on one "
                                        f"thread, {dt1:.2f} s, scaled to N={N} by the point "
                                        "count"}}


def cpu_baseline_configs(args):
    """The cpu_baseline leg over the method's workloads: the FP64 oracle on
    every host thread and on one.  blobs_2k: its whole 500-iteration run
    under the coin with the standard schedule; image_70k (alpha 1): its
    first 100 iterations under the coin (5 on one thread); manifold_1m (FP32
    rows) and zipf_4m (BF16 rows): HD-refining and LD-only iterations after
    an untimed init, on one thread over a uniform sample of the rows (the
    first rows of the shuffled set) scaled to N by the point count.  Each
    timed part prints a progress line to stderr."""
    import numpy as np

    from inputs.generators import RUN_SEED, f32_to_bf16_bits, make_workload, y_init
    from oracle import oracle as O

    threads = O.num_threads()

    def log(msg):
        print(f"[cpu_baseline] {msg}", file=sys.stderr, flush=True)

    def hyper(cfg, N, t, hd_mode):
        early = t < 250
        return O.Hyper(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=float(N / 12.0),
                       momentum=0.5 if early else 0.8, attr=12.0 if early else 1.0,
                       n_neg=cfg["n_neg"], hd_mode=hd_mode)

    def state(X, cfg, Y0):
        N = X.shape[0]
        return O.OracleState(X, cfg["d"], cfg["K_hd"], cfg["K_ld"], RUN_SEED, Y0).init(
            hyper(cfg, N, 0, 0))

    def coin_run(X, cfg, n_iter):
        N = X.shape[0]
        S = state(X, cfg, y_init(N, cfg["d"]))
        fired, t0 = 0, time.perf_counter()
        for t in range(n_iter):
            fired += S.step(hyper(cfg, N, t, 0))["fired"]
        return time.perf_counter() - t0, fired

    def fixed_iters(X, cfg, n_hd, n_ld):
        N = X.shape[0]
        S = state(X, cfg, y_init(N, cfg["d"]))
        t0 = time.perf_counter()
        for t in range(n_hd):
            S.step(hyper(cfg, N, t, 1))
            log(f"  HD-refining iteration {t + 1} of {n_hd} done")
        t1 = time.perf_counter()
        for t in range(n_ld):
            S.step(hyper(cfg, N, n_hd + t, 2))
        t2 = time.perf_counter()
        return (t1 - t0) / max(n_hd, 1), (t2 - t1) / max(n_ld, 1)

    out = {"metric": "oracle seconds per iteration per workload (FP64 C, OpenMP over points)",
           "cores": threads, "workloads": {}}
    W = out["workloads"]
    try:
        # configuration 1: the whole run
        X, _, cfg = make_workload("blobs_2k")
        for nt in (threads, 1):
            O.set_num_threads(nt)
            dt, fired = coin_run(X, cfg, cfg["n_iter"])
            W.setdefault("blobs_2k", {})[f"threads_{nt}"] = {
                "iterations": cfg["n_iter"], "refinements": fired, "seconds": round(dt, 3),
                "s_per_iter": round(dt / cfg["n_iter"], 5)}
            log(f"blobs_2k {nt} threads: {dt:.2f} s")
        # configuration 2 at alpha 1: the first iterations of the run
        X, _, cfg = make_workload("image_70k")
        cfg["alpha"] = 1.0
        for nt, n in ((threads, 100), (1, 5)):
            O.set_num_threads(nt)
            dt, fired = coin_run(X, cfg, n)
            W.setdefault("image_70k", {})[f"threads_{nt}"] = {
                "iterations": n, "refinements": fired, "seconds": round(dt, 3),
                "s_per_iter": round(dt / n, 4)}
            log(f"image_70k {nt} threads: {dt:.2f} s")
        del X
        # configurations 3 and 5: HD-refining and LD-only iterations
        for name, bf16, n_fix, n_one, sample in (("manifold_1m", False, 5, 2, 200_000),
                                                 ("zipf_4m", True, 3, 2, 200_000)):
            X, _, cfg = make_workload(name)
            if bf16:
                X = f32_to_bf16_bits(X)
            N = X.shape[0]
            log(f"{name}: rows ready")
            O.set_num_threads(threads)
            hd, ld = fixed_iters(X, cfg, n_fix, n_fix)
            W[name] = {"rows": "BF16" if bf16 else "FP32", f"threads_{threads}": {
                "hd_iterations": n_fix, "ld_iterations": n_fix, "s_per_hd_iter": round(hd, 3),
                "s_per_ld_iter": round(ld, 3), "points": N}}
            log(f"{name} {threads} threads: HD {hd:.2f} s, LD {ld:.2f} s per iteration")
            O.set_num_threads(1)
            ns = min(sample, N)
            hd1, ld1 = fixed_iters(np.ascontiguousarray(X[:ns]), cfg, n_one, n_one)
            W[name]["threads_1"] = {
                "hd_iterations": n_one, "ld_iterations": n_one, "points": ns,
                "s_per_hd_iter_scaled": round(hd1 * N / ns, 2),
                "s_per_ld_iter_scaled": round(ld1 * N / ns, 2)}
            log(f"{name} 1 thread ({ns} rows): HD {hd1:.2f} s, LD {ld1:.2f} s per iteration")
            del X
    finally:
        O.set_num_threads(threads)
    return out


def feedback_run(F, args):
    """Quality of the HD lists over the iterations with the embedding held
    fixed (learning rate 0: the LD side gives no feedback) and optimised, at
    d = 2 and d = 8 (the feedback-loop experiment of Sec. 3): AUC of
    R_NX(K), K = 1 .. K_hd, of the HD lists against the exact neighbours of a
    query sample, every ``fb_every`` iterations."""
    import numpy as np

    from inputs.generators import RUN_SEED, make_workload, y_init
    from inputs.knn_metrics import exact_knn, rnx_auc, rnx_curve

    X, _, cfg = make_workload("manifold_1m", N=args.fb_n)
    N, K = X.shape[0], args.fb_k
    perp = cfg["perplexity"] if K <= 32 else float(args.fb_perplexity)
    rng = np.random.default_rng(11)
    q = np.sort(rng.choice(N, min(1000, N), replace=False))
    ex, _ = exact_knn(X, q, K)
    out = {"metric": f"HD-list AUC of R_NX(K), K=1..{K}, fixed vs optimised embedding",
           "config": {"workload": f"manifold rows, N={N}, D=128 FP32, K_hd={K}, "
                                  f"K_ld={cfg['K_ld']}, 16 negatives, alpha=1, perplexity {perp}, "
                                  "HD refinement by the coin",
                      "iters": args.fb_iters, "every": args.fb_every, "queries": int(q.size)},
           "curves": {}}
    # jump start: two random projections, each held for js iterations at
    # learning rate 0, then the usual schedule from its beginning
    js = 100
    for d in (2, 8):
        for mode in ("fixed", "optimised", "jumpstart"):
            lr = 0.0 if mode == "fixed" else N / 12.0
            base = dict(alpha=cfg["alpha"], perplexity=perp, lr=lr, n_neg=cfg["n_neg"],
                        hd_mode=0)
            emb = F.Embedding(X, y_init(N, d), d, K, cfg["K_ld"], seed=RUN_SEED,
                              hp=schedule(F, base, 0))
            t0 = 2 * js if mode == "jumpstart" else 0   # where the schedule starts
            curve, done = [], 0
            while True:
                idx, _ = emb.knn(0)
                curve.append([done, round(rnx_auc(rnx_curve(idx[q], ex, N)), 4)])
                if done >= args.fb_iters:
                    break
                n = min(args.fb_every, args.fb_iters - done)
                for edge in (t0 + 250, js, 2 * js):
                    if done < edge < done + n:
                        n = edge - done
                if mode == "jumpstart" and done < 2 * js:
                    if done in (0, js):
                        emb.jump_start(done // js, 1e-2)
                    emb.set_hyperparams(F.fsne_default_hparams(**{**schedule(F, base, 0).as_dict(),
                                                                  "lr": 0.0}))
                else:
                    emb.set_hyperparams(schedule(F, base, done - t0))
                emb.step(n)
                done += n
            emb.close()
            out["curves"][f"d{d}_{mode}"] = curve
    return out


def blobs_knn_run(F, args):
    """Quality of the HD lists on two engineered blob sets (the comparison of
    neighbour finding in Sec. 4.1, without its NN-descent side): 'overlapping',
    5 Gaussian blobs whose centres lie close together against their spread,
    and 'disjointed', 1000 blobs of 30 points far apart against their spread.
    N = 30,000, D = 50, d = 2, K_hd = --fb-k (256 by default), K_ld = 32, 16
    negatives, alpha = 1, perplexity --fb-perplexity (10 for K_hd = 32), the
    standard schedule, the HD refinement by the coin.  R_NX(K), K = 1 .. K_hd,
    of the HD lists against the exact neighbours of 3,000 query points: its
    mean and its spread (standard deviation) across the points, at iterations
    3000 and 9000."""
    import numpy as np

    from inputs.generators import RUN_SEED, blobs, y_init
    from inputs.knn_metrics import exact_knn, rnx_auc, rnx_points

    sets = {"overlapping": dict(n_clusters=5, per_cluster=6000, mean_var=0.25, seed=1021),
            "disjointed": dict(n_clusters=1000, per_cluster=30, mean_var=100.0, seed=1023)}
    Kh = args.fb_k
    perp = 10.0 if Kh <= 32 else float(args.fb_perplexity)
    out = {"metric": "HD-list R_NX(K), mean and spread across points, at 3000 and 9000 iterations",
           "config": {"workload": "Gaussian blobs, N=30,000, D=50 FP32 (overlapping: 5 blobs, "
                                  "centres N(0, 0.25 I); disjointed: 1000 blobs of 30, centres "
                                  f"N(0, 100 I); unit spread in both), d=2, K_hd={Kh}, K_ld=32, "
                                  f"16 negatives, alpha=1, perplexity {perp}, HD refinement by "
                                  "the coin",
                      "queries": 3000},
           "sets": {}}
    for name, kw in sets.items():
        X, _ = blobs(D=50, **kw)
        N = X.shape[0]
        rng = np.random.default_rng(13)
        q = np.sort(rng.choice(N, 3000, replace=False))
        ex, _ = exact_knn(X, q, Kh)
        base = dict(alpha=1.0, perplexity=perp, lr=N / 12.0, n_neg=16, hd_mode=0)
        emb = F.Embedding(X, y_init(N, 2), 2, Kh, 32, seed=RUN_SEED, hp=schedule(F, base, 0))
        res, done, secs = {}, 0, 0.0
        for stop in (250, 3000, 9000):
            emb.sync()
            t0 = time.perf_counter()
            emb.step(stop - done)
            emb.sync()
            secs += time.perf_counter() - t0
            done = stop
            if stop == 250:
                emb.set_hyperparams(schedule(F, base, 250))
                continue
            idx, _ = emb.knn(0)
            pts = rnx_points(idx[q], ex, N)
            mean = pts.mean(axis=0)
            res[str(stop)] = {"seconds": round(secs, 3),
                              "hd_refinements": int(emb.stats()["hd_refinements"]),
                              "rnx_auc": round(rnx_auc(mean), 4),
                              "rnx_mean": [round(float(v), 4) for v in mean],
                              "rnx_std": [round(float(v), 4) for v in pts.std(axis=0)]}
        emb.close()
        out["sets"][name] = res
    return out


def hierarchy_run(F, args):
    """The hierarchy graph of Sec. 4.2 on a two-level Gaussian mixture (4 top
    clusters of 4 sub-clusters, 1000 points each, D = 50) embedded in d = 4:
    after 1000 iterations at alpha = 1, alpha is lowered level by level (the
    LD tails get heavier); at each level the embedding runs 400 iterations
    and is clustered (DBSCAN on the LD lists, min_pts 20, eps twice the
    median distance to the 30th nearest neighbour in the embedding, measured
    on a sample); edges link clusters of consecutive levels with weight
    |A and B| / min(|A|, |B|).  Each level also reports the agreement (ARI)
    of the list-based clusters with exact DBSCAN on the same snapshot."""
    import numpy as np
    from sklearn.cluster import DBSCAN
    from sklearn.metrics import adjusted_rand_score

    from inputs.generators import RUN_SEED, hierarchy_mixture, y_init

    X, top, leaf = hierarchy_mixture()
    N, d, K = X.shape[0], 4, 32
    alphas = [1.0, 0.7, 0.5, 0.35, 0.25, 0.18]
    base = dict(alpha=1.0, perplexity=10.0, lr=N / 12.0, n_neg=16, hd_mode=0)
    emb = F.Embedding(X, y_init(N, d), d, K, K, seed=RUN_SEED, hp=schedule(F, base, 0))
    emb.step(250)
    emb.set_hyperparams(schedule(F, base, 250))
    emb.step(750)
    rng = np.random.default_rng(5)
    sample = rng.choice(N, 2000, replace=False)
    levels, labels = [], []
    for a in alphas:
        emb.set_hyperparams(F.fsne_default_hparams(**{**schedule(F, base, 1000).as_dict(),
                                                      "alpha": a}))
        emb.step(400)
        Y = emb.Y().astype(np.float64)
        d2 = ((Y[sample][:, None, :] - Y[None, :, :]) ** 2).sum(-1)
        kth = np.sqrt(np.sort(d2, axis=1)[:, 30])         # column 0 is the point itself
        eps = float(2.0 * np.median(kth))
        t0 = time.perf_counter()
        lab, nc = emb.cluster(eps, 20)
        ms = (time.perf_counter() - t0) * 1e3
        ok = lab >= 0
        exact = DBSCAN(eps=eps, min_samples=20).fit(Y).labels_
        levels.append({"alpha": a, "eps": round(eps, 4), "clusters": nc,
                       "noise": round(float(1 - ok.mean()), 4),
                       "ari_top": round(adjusted_rand_score(top[ok], lab[ok]), 4),
                       "ari_leaf": round(adjusted_rand_score(leaf[ok], lab[ok]), 4),
                       "exact_dbscan_clusters": int(exact.max() + 1),
                       "ari_vs_exact_dbscan": round(adjusted_rand_score(exact, lab), 4),
                       "cluster_ms": round(ms, 2)})
        labels.append((lab, nc))
    edges = []
    for g in range(len(labels) - 1):
        (la, ca), (lb, cb) = labels[g], labels[g + 1]
        E = F.fsne_hierarchy_edges(la, ca, lb, cb)
        for i, j in zip(*np.nonzero(E >= 0.5)):
            edges.append([g, int(i), g + 1, int(j), round(float(E[i, j]), 3),
                          int((la == i).sum()), int((lb == j).sum())])
    emb.close()
    return {"metric": "alpha-sweep hierarchy graph: clusters per level and edges",
            "config": {"workload": f"two-level Gaussian mixture, N={N}, D=50, 4 x 4 clusters, "
                                   f"d={d}, K_hd=K_ld={K}"},
            "levels": levels, "edges_ge_0.5": edges}


def large_run(F, args):
    """The large BF16 workload: 4,000,000 points of a 1,000-cluster Zipf
    mixture in R^256 (BF16 rows), d = 32, K_hd = 64, K_ld = 32, 32 negatives,
    alpha = 0.5, perplexity 20.  Reports the step time with the HD refinement
    on and off (and with the BF16 MFMA screen), the per-kernel times, and
    500-iteration runs, under the coin and with every iteration refining, each
    also with the points renumbered for locality every 100 iterations, with
    HD recall@64 of 500 query points against exact neighbours."""
    import numpy as np
    import torch

    from inputs.generators import RUN_SEED, bf16_bits_to_f32, f32_to_bf16_bits, make_workload, y_init
    from inputs.knn_metrics import exact_knn_device, recall_at_k

    t_gen = time.perf_counter()
    X, _, cfg = make_workload("zipf_4m")
    Xb = f32_to_bf16_bits(X)
    del X
    t_gen = time.perf_counter() - t_gen
    N, K = Xb.shape[0], cfg["K_hd"]
    Y0 = y_init(N, cfg["d"])
    base = dict(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N / 12.0,
                n_neg=cfg["n_neg"], dist_mode=0)
    out = {"metric": "large BF16 workload: iters/s and HD recall@64",
           "config": {"workload": "zipf_4m: N=4,000,000 points of a 1000-cluster Zipf(1.1) mixture "
                                  "in R^256 (BF16 rows), d=32, K_hd=64, K_ld=32, 32 negatives, "
                                  "alpha=0.5, perplexity 20"},
           "data_gen_seconds": round(t_gen, 1)}
    for mode, dm, name in ((1, 0, "hd_always"), (2, 0, "ld_only"), (1, 1, "hd_always_mfma_screen")):
        emb = F.Embedding(Xb, Y0, cfg["d"], K, cfg["K_ld"], seed=RUN_SEED,
                          hp=F.fsne_default_hparams(**{**schedule(F, base, 0).as_dict(),
                                                       "hd_mode": mode, "dist_mode": dm}))
        if args.reorder_data:
            emb.reorder_data()
        emb.step(5)
        emb.sync()
        t0 = time.perf_counter()
        emb.step(20)
        emb.sync()
        ms = (time.perf_counter() - t0) * 1e3 / 20
        emb.profile(True)
        emb.step(10)
        kt = emb.kernel_times()
        emb.close()
        out[name] = {"ms_per_step": round(ms, 3), "iters_per_s": round(1e3 / ms, 2),
                     "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]}}
    if args.large_steps_only:
        return out
    rng = np.random.default_rng(7)
    q = np.sort(rng.choice(N, 500, replace=False))
    Xd = torch.from_numpy(bf16_bits_to_f32(Xb)).cuda()
    _, ex = exact_knn_device(Xd, Xb, q, K)
    del Xd
    torch.cuda.empty_cache()
    # 500 iterations under the coin, then the same with every iteration
    # refining; each also with the points renumbered along the embedding's
    # Morton order every 100 iterations (timed; the lists are mapped back to
    # the original ids to be measured)
    runs = [(0, "run_500", 0), (1, "run_500_hd_always", 0)]
    if args.reorder_every > 0:
        runs += [(0, "run_500_renumbered", 100), (1, "run_500_hd_always_renumbered", 100)]
    for hd_mode, name, every in runs:
        emb = F.Embedding(Xb, Y0, cfg["d"], K, cfg["K_ld"], seed=RUN_SEED,
                          hp=schedule(F, {**base, "hd_mode": hd_mode}, 0))
        emb.sync()
        orig = np.arange(N)
        t0 = time.perf_counter()
        if args.reorder_data:
            track_renumbering(orig, emb.reorder_data())
        for done in range(0, 500, 100):
            if every and done > 0:
                track_renumbering(orig, emb.reorder())
            if done < 250 < done + 100:
                emb.step(250 - done)
                emb.set_hyperparams(schedule(F, {**base, "hd_mode": hd_mode}, 250))
                emb.step(done + 100 - 250)
            else:
                emb.step(100)
        emb.sync()
        secs = time.perf_counter() - t0
        idx = emb.knn(0)[0]
        lists = np.empty_like(idx)
        lists[orig] = orig[idx]
        st = emb.stats()
        emb.close()
        out[name] = {"seconds": round(secs, 3), "iters_per_s": round(500 / secs, 2),
                     "recall_at_64": round(recall_at_k(lists, Xb, q, ex), 4),
                     "final_E": round(float(st["E"]), 4), "nonfinite": int(st["nonfinite"])}
    return out


def image_run(F, args):
    """The image-like workload: 70,000 rows of 784 values in [0, 1] (about 80 %
    zeros) from 10 class prototypes, FP32, embedded in 2-D with K_hd = K_ld =
    32, 16 negatives, perplexity 10, for each tail alpha in {0.5, 1, 4}:
    2000 iterations under the coin with the standard schedule (learning rate
    N/48, as for the 2-D online-use runs), wall seconds, HD recall@32 on
    1,000 queries against exact neighbours, and the fraction of each point's
    32 LD neighbours that share its class."""
    import numpy as np

    from inputs.generators import RUN_SEED, make_workload, y_init
    from inputs.knn_metrics import exact_knn

    X, lab, cfg = make_workload("image_70k")
    N, K = X.shape[0], cfg["K_hd"]
    rng = np.random.default_rng(3)
    q = np.sort(rng.choice(N, 1000, replace=False))
    _, ex = exact_knn(X, q, K)
    out = {"metric": "iters/s and HD recall@32 per tail alpha",
           "config": {"workload": "image_70k: N=70,000 image-like rows in [0,1]^784 (FP32), d=2, "
                                  "K_hd=K_ld=32, 16 negatives, perplexity 10, 2000 iterations",
                      "queries": int(q.size), "lr": "N/48"},
           "alphas": {}}
    for alpha in cfg["alpha"]:
        cfg_a = {**cfg, "alpha": alpha}
        r = quality_run(F, X, cfg_a, y_init(N, 2), cfg["n_iter"], RUN_SEED, q, ex, every=500,
                        labels=lab, lr_div=48.0)
        out["alphas"][str(alpha)] = r
    return out


def memo_run(F, args):
    """The memory of rejected HD candidates off and on: with every iteration
    refining and the standard schedule, the HD kernel's time and the candidate
    rows read per point, averaged over the 10 iterations ending at iterations
    35, 120 and 320, for the 1M manifold (FP32, 512-byte rows), the 70k
    image-like (FP32, 3136-byte rows, alpha 1) and the 4M Zipf (BF16, 512-byte
    rows, K_hd = 64) workloads.  Both settings give the same lists and
    embedding bit for bit; only the rows read and the time differ."""
    import numpy as np

    from inputs.generators import RUN_SEED, f32_to_bf16_bits, make_workload, y_init

    out = {"metric": "HD kernel ms and candidate rows per point, memory of rejections off/on",
           "workloads": {}}
    for name in ("manifold_1m", "image_70k", "zipf_4m"):
        X, _, cfg = make_workload(name)
        if name == "zipf_4m":
            X = f32_to_bf16_bits(X)
        alpha = 1.0 if isinstance(cfg["alpha"], (list, tuple)) else cfg["alpha"]
        N = X.shape[0]
        Y0 = y_init(N, cfg["d"])
        base = dict(alpha=alpha, perplexity=cfg["perplexity"],
                    lr=N / (48.0 if cfg["d"] == 2 else 12.0), n_neg=cfg["n_neg"], hd_mode=1)
        res = {}
        for memo in (0, 1):
            def hp(t):
                return F.fsne_default_hparams(**{**schedule(F, base, t).as_dict(),
                                                 "reject_memo": memo})
            emb = F.Embedding(X, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hp(0))
            t, pts = 0, []
            for stop in (25, 110, 310):
                if t < 250 <= stop:
                    emb.step(250 - t)
                    t = 250
                    emb.set_hyperparams(hp(250))
                emb.step(stop - t)
                t = stop
                emb.profile(True)
                rows = []
                for _ in range(10):
                    emb.step(1)
                    rows.append(emb.stats()["hd_cand_rows"] / N)
                t += 10
                kt = emb.kernel_times()
                emb.profile(False)
                ms, n = kt["hd_refine"]
                pts.append({"iteration": t, "hd_refine_ms": round(ms / max(n, 1), 4),
                            "rows_per_point": round(float(np.mean(rows)), 2)})
            emb.close()
            res["on" if memo else "off"] = pts
        out["workloads"][name] = {"N": int(N), "D": int(X.shape[1]),
                                  "dtype": "bf16" if X.dtype == np.uint16 else "f32",
                                  "K_hd": cfg["K_hd"], **res}
        del X
    return out


def scaling_run(F, args):
    """Time per iteration across dataset sizes at a fixed input dimensionality
    of 32 (the setting of the paper's timing figure, Sec. 4): manifold rows
    (50 linear 8-dim manifolds in R^32, FP32), d = 2, K_hd = K_ld = 32, 16
    negatives, alpha = 1, perplexity 10.  For each N: ms per iteration with
    the HD refinement on every step and with it off, and the mean over a
    500-iteration run under the coin with the standard schedule, also with
    the points renumbered every 100 iterations."""
    from inputs.generators import RUN_SEED, manifolds, y_init

    out = {"metric": "ms per iteration vs N at D = 32",
           "config": {"workload": "manifold rows, 50 linear 8-dim manifolds in R^32 (FP32), d=2, "
                                  "K_hd=K_ld=32, 16 negatives, alpha=1, perplexity 10"},
           "sizes": []}
    for N in args.scaling_sizes:
        X, _ = manifolds(n_manifolds=50, per_manifold=N // 50, D=32)
        N = X.shape[0]
        Y0 = y_init(N, 2)
        base = dict(alpha=1.0, perplexity=10.0, lr=N / 12.0, n_neg=16)
        row = {"N": N}
        for mode, name in ((1, "hd_always_ms"), (2, "ld_only_ms")):
            emb = F.Embedding(X, Y0, 2, 32, 32, seed=RUN_SEED,
                              hp=schedule(F, {**base, "hd_mode": mode}, 0))
            emb.step(10)
            emb.sync()
            t0 = time.perf_counter()
            emb.step(50)
            emb.sync()
            row[name] = round((time.perf_counter() - t0) * 1e3 / 50, 4)
            emb.close()
        emb = F.Embedding(X, Y0, 2, 32, 32, seed=RUN_SEED, hp=schedule(F, {**base, "hd_mode": 0}, 0))
        emb.sync()
        t0 = time.perf_counter()
        emb.step(250)
        emb.set_hyperparams(schedule(F, {**base, "hd_mode": 0}, 250))
        emb.step(250)
        emb.sync()
        row["run_500_mean_ms"] = round((time.perf_counter() - t0) * 1e3 / 500, 4)
        emb.close()
        if args.reorder_every > 0:
            # the same run with the points renumbered every 100 iterations (timed)
            emb = F.Embedding(X, Y0, 2, 32, 32, seed=RUN_SEED,
                              hp=schedule(F, {**base, "hd_mode": 0}, 0))
            emb.sync()
            t0 = time.perf_counter()
            for done in range(0, 500, 100):
                if done:
                    emb.reorder()
                if done < 250 < done + 100:
                    emb.step(250 - done)
                    emb.set_hyperparams(schedule(F, {**base, "hd_mode": 0}, 250))
                    emb.step(done + 100 - 250)
                else:
                    emb.step(100)
            emb.sync()
            row["run_500_renumbered_mean_ms"] = round((time.perf_counter() - t0) * 1e3 / 500, 4)
            emb.close()
        out["sizes"].append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return out


STEP_KERNELS = (("hd_refine", "k_hd_refine"), ("affinity", "k_psym"), ("ld_grad", "k_ld_grad"),
                ("reduce", "k_reduce"), ("update", "k_update"))


def counted_traffic(kernel, W, K, reorder):
    """HBM bytes per launch of `kernel` in the timed iterations, from
    profiles/traffic.json, if it was taken with the current step sources over
    the same iterations and renumbering (else None)."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    recs = json.load(open(tf))
    for rec in (recs if isinstance(recs, list) else [recs]):
        if (rec.get("source_hash") == kernel_source_hash() and rec.get("window") == [W, K]
                and rec.get("reorder") == list(reorder)):
            return rec.get("per_launch_GB", {}).get(kernel)
    return None


def roofline(kernels, name, W, K, reorder):
    """The roofline object of the dominant kernel.  achieved = its algorithmic
    bytes per launch over its average launch duration.  Where that exceeds the
    HBM peak (renumbered points: the caches serve part of the bytes) the
    fraction of HBM is taken from the counted HBM traffic of the same
    iterations instead, and the share the caches served is stated."""
    k = kernels[name]
    avg_s = k["avg_ms"] * 1e-3
    traffic = counted_traffic(name, W, K, reorder)
    r = {"bound": "hbm", "kernel": name, "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "algorithmic_GB_per_launch": k["algorithmic_GB"], "avg_launch_ms": k["avg_ms"],
         "traffic": traffic,
         "traffic_unit": "GB per launch (FETCH_SIZE x2 + WRITE_SIZE x1, calibrated on a copy)"}
    if k["GBps"] <= PEAK_HBM_GBS:
        r.update(achieved=k["GBps"], frac=round(k["GBps"] / PEAK_HBM_GBS, 4),
                 basis="algorithmic bytes per launch / average launch duration")
    elif traffic is not None:
        ach = traffic / avg_s
        r.update(achieved=round(ach, 1), frac=round(ach / PEAK_HBM_GBS, 4),
                 algorithmic_GBps=k["GBps"],
                 cache_served=round(1.0 - traffic / k["algorithmic_GB"], 4),
                 basis="counted HBM bytes per launch / average launch duration: the "
                       "algorithmic bytes exceed what HBM moves in that time, the caches "
                       "serve the rest")
    else:
        r.update(achieved=None, frac=None, algorithmic_GBps=k["GBps"],
                 basis="the algorithmic bytes exceed what HBM moves in the launch time (the "
                       "caches serve part) and no counted traffic matches these sources")
    if traffic is not None:
        r["traffic_GBps"] = round(traffic / avg_s, 1)
        r["traffic_frac"] = round(traffic / avg_s / PEAK_HBM_GBS, 4)
    return r


def bf16_error_statement(F, X, Xb, emb, cfg, n_points=2000, seed=11):
    """Per-result error of the BF16 form: the stored HD distances (FP32 re-rank
    of BF16 rows) against exact FP64 distances of the same BF16 rows and of
    the original FP32 rows, on a sample of points; and the neighbours the MFMA
    screen loses in one refinement against direct distances from the same
    state."""
    import numpy as np

    from inputs.generators import RUN_SEED, bf16_bits_to_f32

    g = emb.state()
    N = Xb.shape[0]
    pts = np.sort(np.random.default_rng(seed).choice(N, n_points, replace=False))
    Xbf = bf16_bits_to_f32(Xb)
    idx, d2 = g["hd_idx"][pts], g["hd_d2"][pts].astype(np.float64)
    e_b = ((Xbf[idx].astype(np.float64) - Xbf[pts][:, None, :].astype(np.float64)) ** 2).sum(-1)
    e_f = ((X[idx].astype(np.float64) - X[pts][:, None, :].astype(np.float64)) ** 2).sum(-1)
    rb = np.abs(d2 - e_b) / np.maximum(e_b, 1e-30)
    rf = np.abs(d2 - e_f) / np.maximum(e_f, 1e-30)
    q = lambda a: {"median": float(f"{np.median(a):.3g}"), "p99": float(f"{np.quantile(a, 0.99):.3g}"),
                   "max": float(f"{a.max():.3g}")}
    # one refinement from the same state, screened and direct
    lists = {}
    for dm in (0, 1):
        hpf = F.fsne_default_hparams(**{**emb.hyperparams().as_dict(), "dist_mode": dm,
                                        "hd_mode": 1})
        e = F.Embedding(Xb, g["Y"], cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hpf)
        e.set_state({k: v for k, v in g.items() if k not in ("A", "R", "Zh")})
        e.step(1)
        lists[dm] = e.knn(0)[0]
        e.close()
    diff = lists[0] != lists[1]
    rows = np.nonzero(diff.any(1))[0]
    lost = sum(len(set(lists[0][i].tolist()) - set(lists[1][i].tolist())) for i in rows)
    return {"points": int(n_points),
            "rel_err_vs_fp64_of_bf16_rows": q(rb),
            "rel_err_vs_fp64_of_fp32_rows": q(rf),
            "screen_lost_neighbours_one_refinement": int(lost),
            "screen_rows_differing": int(rows.size),
            "screen_lost_per_point": float(f"{lost / N:.3g}")}


def summarize_profile(args):
    """Figures of the timed iterations from rocprofv3 CSV output: the step
    kernels' dispatches are assigned to iterations (one k_update ends each,
    the last dispatch of a kernel before it is the step's), and those of
    iterations warmup .. warmup+steps-1 of the first embedding are averaged.
    Directories given as name=dir: 'trace' (kernel trace: microseconds),
    others (counter collection: KiB per dispatch, instances summed); 'cfetch'
    and 'cwrite' are the copy-probe runs that calibrate FETCH_SIZE and
    WRITE_SIZE."""
    import csv
    import glob
    from collections import defaultdict

    W, K = args.warmup, args.steps
    out = {"window": [W, K],
           "reorder": [args.reorder_every, args.reorder_from, int(args.reorder_data)]}
    dirs = dict(x.split("=", 1) for x in args.summarize_profile)

    def rows_of(d, pattern):
        files = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
        assert files, f"no {pattern} under {d}"
        rows = []
        for fn in files:
            with open(fn) as fh:
                rows += list(csv.DictReader(fh))
        return rows

    def per_iteration(disp):
        """disp: [(dispatch id, kernel name, value)] -> {kernel: [value per iteration]}."""
        it, cur, per = 0, {}, defaultdict(list)
        for _, kname, v in sorted(disp):
            for key, pat in STEP_KERNELS:
                if pat in kname:
                    cur[key] = v
                    if key == "update":
                        for kk, vv in cur.items():
                            per[kk].append((it, vv))
                        it, cur = it + 1, {}
        return {k: [v for i, v in lst if W <= i < W + K] for k, lst in per.items()}

    for name, d in dirs.items():
        if name == "trace":
            rows = rows_of(d, "*kernel_trace.csv")
            disp = [(int(r["Dispatch_Id"]), r["Kernel_Name"],
                     (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3) for r in rows]
            per = per_iteration(disp)
            out["trace_us"] = {k: {"launches": len(v), "avg_us": round(sum(v) / len(v), 1),
                                   "min_us": round(min(v), 1), "max_us": round(max(v), 1)}
                               for k, v in per.items() if v}
        else:
            rows = rows_of(d, "*counter_collection.csv")
            acc = defaultdict(float)
            names = {}
            for r in rows:
                key = (int(r["Dispatch_Id"]), r["Counter_Name"])
                acc[key] += float(r["Counter_Value"])
                names[key[0]] = r["Kernel_Name"]
            counters = sorted({c for _, c in acc})
            for c in counters:
                disp = [(di, names[di], v) for (di, cc), v in acc.items() if cc == c]
                if name in ("cfetch", "cwrite"):
                    biggest = max(v for _, _, v in disp)
                    out[f"{name}_{c}_KiB"] = biggest
                    continue
                per = per_iteration(disp)
                out.setdefault("counters_KiB", {})[c] = {
                    k: round(sum(v) / len(v), 1) for k, v in per.items() if v}
    if "cfetch" in dirs and "cwrite" in dirs and "counters_KiB" in out:
        copy_kib = args.copy_bytes / 1024.0
        f_fetch = round(copy_kib / out["cfetch_FETCH_SIZE_KiB"], 2)
        f_write = round(copy_kib / out["cwrite_WRITE_SIZE_KiB"], 2)
        c = out["counters_KiB"]
        per_launch = {k: round((c["FETCH_SIZE"][k] * f_fetch + c["WRITE_SIZE"][k] * f_write)
                               * 1024 / 1e9, 3)
                      for k in c["FETCH_SIZE"] if k in c.get("WRITE_SIZE", {})}
        out["factors"] = {"FETCH_SIZE": f_fetch, "WRITE_SIZE": f_write}
        out["per_launch_GB"] = per_launch
        if args.write_traffic:
            # one record per (window, renumbering policy, sources); others are kept
            rec = {"source_hash": kernel_source_hash(), "workload": "manifold_1m",
                   "window": [W, K], "reorder": out["reorder"],
                   "unit": "GB per launch", "factors": out["factors"],
                   "per_launch_GB": per_launch, "sources": list(STEP_SOURCES)}
            tf = os.path.join(ROOT, "profiles", "traffic.json")
            old = json.load(open(tf)) if os.path.exists(tf) else []
            old = [r for r in (old if isinstance(old, list) else [old])
                   if r.get("source_hash") == rec["source_hash"]
                   and (r.get("window"), r.get("reorder")) != (rec["window"], rec["reorder"])]
            with open(tf, "w") as fh:
                json.dump(old + [rec], fh, indent=1)
    print(json.dumps(out, indent=1))


def summarize_phases(d):
    """Per-embedding figures from rocprofv3 output of a command that builds
    several embeddings one after another (`--large`): the dispatches are split
    into phases at each launch of the list initialisation, and for every
    phase each step kernel's launches and its mean over all of them and over
    the last 10 are printed: durations in microseconds from a kernel trace,
    or each counter (summed over its instances) from a counter collection."""
    import csv
    import glob
    from collections import defaultdict

    def rows_of(pattern):
        rows = []
        for fn in sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True)):
            with open(fn) as fh:
                rows += list(csv.DictReader(fh))
        return rows

    trace = rows_of("*kernel_trace.csv")
    if trace:
        disp = {int(r["Dispatch_Id"]): (r["Kernel_Name"], {
            "us": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3}) for r in trace}
    else:
        disp = {}
        for r in rows_of("*counter_collection.csv"):
            k = int(r["Dispatch_Id"])
            name, vals = disp.setdefault(k, (r["Kernel_Name"], defaultdict(float)))
            vals[r["Counter_Name"]] += float(r["Counter_Value"])
    assert disp, f"no kernel trace or counter collection under {d}"
    phases, cur = [], None
    for k in sorted(disp):
        kname, vals = disp[k]
        if "k_init_lists" in kname:
            cur = defaultdict(list)
            phases.append(cur)
            continue
        if cur is None:
            continue
        for key, pat in STEP_KERNELS:
            if pat in kname:
                cur[key].append(vals)
    out = []
    for k, ph in enumerate(phases):
        rec = {"phase": k}
        for key, lst in ph.items():
            names = sorted(lst[0])
            rec[key] = {"launches": len(lst),
                        **{f"mean_{n}": round(sum(v[n] for v in lst) / len(lst), 1) for n in names},
                        **{f"last10_{n}": round(sum(v[n] for v in lst[-10:]) / len(lst[-10:]), 1)
                           for n in names}}
        out.append(rec)
    print(json.dumps(out, indent=1))


def mlp_flops(D, H1, H2, d, n):
    """Multiply-add flops of one training pass over n rows: the forward pass,
    the weight gradients of all three layers and the input gradients of the
    two upper layers."""
    fwd = 2 * n * (D * H1 + H1 * H2 + H2 * d)
    bwd = 2 * n * (D * H1 + 2 * H1 * H2 + 2 * H2 * d)
    return fwd + bwd


def mlp_train_run(F, args):
    """Training time of the placement network alone (784 -> 512 -> 512 -> 2,
    default options: 5 epochs, batches of 4096, Adam) on the online-use
    workload's 500,000 styled image-like rows, with targets from the
    embedding's initial placement (the time does not depend on them); two
    trainings from a new network each."""
    import numpy as np
    import torch

    from inputs.generators import CONFIGS, RUN_SEED, image_styles, y_init

    cfg = CONFIGS["dynamic_500k"]
    N0 = cfg["N"]
    rng = np.random.default_rng(cfg["data_seed"] + 11)
    X, _ = image_styles(rng.permutation(np.arange(N0) % 10), seed=cfg["data_seed"],
                        proto_seed=CONFIGS["image_70k"]["data_seed"])
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N0 / 48.0, n_neg=16)
    emb = F.Embedding(X, y_init(N0, cfg["d"]), cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED,
                      hp=hp)
    o = F.fsne_mlp_default_opts()
    flops = o.epochs * mlp_flops(X.shape[1], o.hidden1, o.hidden2, cfg["d"], N0)
    out = {"metric": "placement network training seconds", "config": {
        "workload": "500,000 styled image-like rows, 784 -> 512 -> 512 -> 2, 5 epochs, "
                    "batches of 4096"}, "runs": []}
    for _ in range(2):
        net = F.Mlp(emb, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.train(emb)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        net.close()
        out["runs"].append({"seconds": round(t, 4), "TFLOPps": round(flops / t / 1e12, 1)})
    emb.close()
    out["library_products"] = library_products(X.shape[1], o.hidden1, o.hidden2, o.batch)
    return out


def library_products(D, H1, H2, B, reps=200):
    """For comparison only: the network's five products of one batch as plain
    library products (torch.mm on BF16 operands, which ROCm serves with
    hipBLASLt), without the fused bias, ReLU, mask and column sums, timed with
    events over back-to-back calls; and one large square product to show the
    library's rate where the shape allows it."""
    import torch

    dev = "cuda"
    g = torch.Generator(device=dev).manual_seed(5)

    def rnd(*shape):
        return torch.randn(*shape, device=dev, dtype=torch.bfloat16, generator=g)

    X, H1m, dH2, dH1 = rnd(B, D), rnd(B, H1), rnd(B, H2), rnd(B, H1)
    W1t, W2t, W2 = rnd(D, H1), rnd(H1, H2), rnd(H2, H1)
    dH2t, dH1t = dH2.t().contiguous(), dH1.t().contiguous()
    S = rnd(8192, 8192)
    cases = [
        (f"H1 = X W1^T ({B} x {H1} x {D})", lambda: torch.mm(X, W1t), 2 * B * H1 * D),
        (f"H2 = H1 W2^T ({B} x {H2} x {H1})", lambda: torch.mm(H1m, W2t), 2 * B * H2 * H1),
        (f"W2 gradient dH2^T H1 ({H2} x {H1} x {B})", lambda: torch.mm(dH2t, H1m),
         2 * B * H2 * H1),
        (f"dH1 = dH2 W2 ({B} x {H1} x {H2})", lambda: torch.mm(dH2, W2), 2 * B * H2 * H1),
        (f"W1 gradient dH1^T X ({H1} x {D} x {B})", lambda: torch.mm(dH1t, X), 2 * B * H1 * D),
        ("square 8192 x 8192 x 8192", lambda: torch.mm(S, S), 2 * 8192 ** 3),
    ]
    res = []
    for name, fn, fl in cases:
        n = 20 if name.startswith("square") else reps
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / n * 1e3
        res.append({"product": name, "us": round(us, 2), "TFLOPps": round(fl / us / 1e6, 1)})
    return res


def dynamic_run(F, args):
    """Online use with learned placement.

    A 500,000-point image-like set is embedded in 2-D (250 iterations with
    attraction 12 and momentum 0.5, then attraction 1 and momentum 0.8), the
    placement network 784-512-512-2 is trained on its (x, y) pairs, and then
    batches of 50,000 new points arrive while 1 % of the live points drift
    (their x is redrawn from a uniformly chosen class).  Two tracks start from
    the same base state: in one the network places the new and drifted points,
    in the other new points start at N(0, 1e-4) and drifted points keep their
    y.  After each batch the step runs in chunks of 10 iterations until the LD
    neighbour recall of a sample of the batch's new points (the fraction of
    their exact 32 HD neighbours among their exact 32 LD neighbours) reaches
    0.9 times the base points' value, or a cap.  Reported per batch and in
    total: iterations and step seconds (evaluation excluded)."""
    import numpy as np
    import torch

    from inputs.generators import CONFIGS, RUN_SEED, image_like, image_styles, y_init
    from inputs.knn_metrics import knn_on_device, set_recall

    cfg = CONFIGS["dynamic_500k"]
    proto = CONFIGS["image_70k"]["data_seed"]

    def rows(classes, seed):
        if args.dyn_data == "styles":
            return image_styles(classes, seed=seed, proto_seed=proto)
        return image_like(classes=classes, seed=seed, proto_seed=proto)

    N0 = args.dyn_base if args.dyn_base else cfg["N"]
    nb, bs, dfrac = args.dyn_batches, cfg["batch_size"], cfg["drift_frac"]
    if args.dyn_base:
        bs = max(1000, N0 // 10)
    K, d = cfg["K_ld"], cfg["d"]
    cap = N0 + nb * bs
    rng = np.random.default_rng(cfg["data_seed"] + 11)
    t_gen = time.perf_counter()
    Xb, lab0 = rows(rng.permutation(np.arange(N0) % 10), cfg["data_seed"])
    labels = np.zeros(cap, np.int32)
    labels[:N0] = lab0
    batches, n_live = [], N0
    for b in range(nb):
        Xn, ln = rows(rng.integers(0, 10, bs), cfg["data_seed"] + 100 + b)
        nd = int(round(dfrac * n_live))
        ids = np.sort(rng.choice(n_live, nd, replace=False)).astype(np.int64)
        Xd, ld = rows(rng.integers(0, 10, nd), cfg["data_seed"] + 200 + b)
        sample = n_live + np.sort(rng.choice(bs, min(1000, bs), replace=False))
        labels[n_live:n_live + bs] = ln
        labels[ids] = ld
        batches.append((Xn, ids, Xd, sample, labels[:n_live + bs].copy()))
        n_live += bs
    t_gen = time.perf_counter() - t_gen

    dev = torch.device("cuda")
    # lr = N/48: in 2-D without per-parameter gains, N/12 lets the sampled
    # far-field repulsion diffuse points out of their classes at this size
    hp = F.fsne_default_hparams(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N0 / 48.0,
                                momentum=0.5, attr=12.0, n_neg=cfg["n_neg"], hd_mode=0)
    hp2 = F.fsne_default_hparams(**{**hp.as_dict(), "attr": 1.0, "momentum": 0.8})
    base = F.Embedding(Xb, y_init(N0, d), d, cfg["K_hd"], K, seed=RUN_SEED, hp=hp,
                       capacity=cap)
    base.sync()
    t0 = time.perf_counter()
    base.step(250)
    base.set_hyperparams(hp2)
    base.step(args.dyn_base_iters - 250)
    base.sync()
    t_base = time.perf_counter() - t0
    snap = {k: v for k, v in base.state().items() if k not in ("A", "R", "Zh")}
    Ybase = base.Y()

    net = F.Mlp(base, F.fsne_mlp_default_opts())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = net.train(base)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    progress(f"online use ({args.dyn_data}): base embedded, network trained")
    o = F.fsne_mlp_default_opts()
    flops = o.epochs * mlp_flops(Xb.shape[1], o.hidden1, o.hidden2, d, N0)

    Xlive = torch.zeros((cap, Xb.shape[1]), dtype=torch.float32, device=dev)
    Xlive[:N0] = torch.from_numpy(Xb).to(dev)
    rows_b = np.sort(rng.choice(N0, 1000, replace=False))
    hd_b = knn_on_device(Xlive[:N0], rows_b, K)
    ld_b = knn_on_device(torch.from_numpy(Ybase).to(dev), rows_b, K, direct=True)
    base_recall = set_recall(hd_b, ld_b)
    base_class = float((lab0[ld_b] == lab0[rows_b][:, None]).mean())
    target = 0.9 * base_recall
    truth, n_live = [], N0
    for Xn, ids, Xd, sample, _ in batches:
        Xlive[n_live:n_live + bs] = torch.from_numpy(Xn).to(dev)
        Xlive[torch.from_numpy(ids).to(dev)] = torch.from_numpy(Xd).to(dev)
        n_live += bs
        truth.append(knn_on_device(Xlive[:n_live], sample, K))
    del Xlive
    torch.cuda.empty_cache()

    tracks = {}
    for mode in ("mlp", "random"):
        emb = F.Embedding(Xb, Ybase, d, cfg["K_hd"], K, seed=RUN_SEED, hp=hp2, capacity=cap)
        emb.set_state(snap)
        res = []
        if mode == "mlp":
            # one more epoch on the live points before each batch keeps the
            # network in step with the embedding as it moves
            ft = F.Mlp(emb, F.fsne_mlp_default_opts(epochs=1))
            ft.set_params(*net.params())
        for b, (Xn, ids, Xd, sample, lab) in enumerate(batches):
            progress(f"online use ({args.dyn_data}, {mode} placement): batch {b}")
            place = 0.0
            if mode == "mlp":
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if b > 0:
                    ft.train(emb)
                Yn, Ydr = ft.predict(Xn), ft.predict(Xd)
                torch.cuda.synchronize()
                place = time.perf_counter() - t0
                emb.insert(Xn, Yn)
                emb.drift(ids, Xd, Ydr)
            else:
                emb.insert(Xn, y_init(bs, d, seed=RUN_SEED + 1000 + b))
                emb.drift(ids, Xd, None)
            it, secs, r0, r, c0 = 0, 0.0, None, 0.0, None
            while True:
                Yd = torch.from_numpy(emb.Y()).to(dev)
                ld_nn = knn_on_device(Yd, sample, K, direct=True)
                r = set_recall(truth[b], ld_nn)
                cls = float((lab[ld_nn] == lab[sample][:, None]).mean())
                if r0 is None:
                    r0, c0 = r, cls
                if r >= target or it >= args.dyn_cap:
                    break
                emb.sync()
                t0 = time.perf_counter()
                emb.step(10)
                emb.sync()
                secs += time.perf_counter() - t0
                it += 10
            res.append({"batch": b, "reached": bool(r >= target), "iters": it,
                        "seconds": round(secs, 4), "placement_seconds": round(place, 4),
                        "recall_at_placement": round(r0, 4),
                        "recall_final": round(r, 4), "same_class_at_placement": round(c0, 4),
                        "same_class_final": round(cls, 4)})
        st = emb.stats()
        if mode == "mlp":
            ft.close()
        tracks[mode] = {"batches": res, "total_iters": sum(x["iters"] for x in res),
                        "total_seconds": round(sum(x["seconds"] for x in res), 3),
                        "total_placement_seconds": round(sum(x["placement_seconds"] for x in res), 3),
                        "all_reached": all(x["reached"] for x in res),
                        "nonfinite": int(st["nonfinite"])}
        emb.close()
    net.close()
    base.close()
    out = {"metric": "dynamic placement: iterations and seconds to LD recall target, "
                     "network vs random placement",
           "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"{args.dyn_data} image-like 784-dim rows, base N={N0}, {nb} "
                                  f"batches of {bs} new points + {dfrac:.0%} drift, d={d}, K={K}",
                      "base_iters": args.dyn_base_iters, "cap_iters": args.dyn_cap},
           "data_gen_seconds": round(t_gen, 1), "base_seconds": round(t_base, 3),
           "mlp_train": {"seconds": round(t_train, 3), "final_loss": round(loss, 5),
                         "flops": flops, "TFLOPps": round(flops / t_train / 1e12, 2),
                         "peak_bf16_TFLOPps": 2500.0},
           "base_ld_recall": round(base_recall, 4), "base_same_class": round(base_class, 4),
           "target": round(target, 4),
           "tracks": tracks}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--quality-iters", type=int, default=1000)
    ap.add_argument("--queries", type=int, default=1000)
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-configs", action="store_true",
                    help="the CPU baseline (FP64 oracle) over every workload, alone")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device to device (counter calibration)")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the online-use experiment")
    ap.add_argument("--feedback", action="store_true",
                    help="run the feedback-loop experiment (fixed vs optimised embedding) instead")
    ap.add_argument("--hierarchy", action="store_true",
                    help="run the alpha-sweep hierarchy graph experiment instead")
    ap.add_argument("--image", action="store_true",
                    help="the 70k image-like workload for tail alphas 0.5, 1, 4")
    ap.add_argument("--scaling", action="store_true",
                    help="time per iteration across N at D = 32 (the paper's timing figure)")
    ap.add_argument("--scaling-sizes", type=int, nargs="+",
                    default=[10_000, 30_000, 100_000, 300_000, 1_000_000, 3_000_000])
    ap.add_argument("--large", action="store_true",
                    help="run the 4M-point BF16 workload instead")
    ap.add_argument("--mlp-train", action="store_true",
                    help="time the placement network's training alone")
    ap.add_argument("--large-steps-only", action="store_true",
                    help="with --large: only the step timings (no 500-iteration runs)")
    ap.add_argument("--reorder-every", type=int, default=25,
                    help="renumber the points along the embedding's Morton order every this "
                         "many steps in the timed runs (0: never)")
    ap.add_argument("--reorder-from", type=int, default=50,
                    help="first iteration before which the timed runs renumber")
    ap.add_argument("--reorder-data", type=int, default=1,
                    help="1: renumber the points along a fixed projection of the data rows "
                         "before iteration 0 (set-up, untimed); 0: keep the input order")
    ap.add_argument("--blobs-knn", action="store_true",
                    help="HD-list R_NX(K) on overlapping and disjointed blobs instead")
    ap.add_argument("--memo-compare", action="store_true",
                    help="HD kernel with the memory of rejected candidates off and on instead")
    ap.add_argument("--summarize-phases", metavar="DIR",
                    help="per-embedding step-kernel durations from a rocprofv3 kernel trace")
    ap.add_argument("--summarize-profile", nargs="+", metavar="NAME=DIR",
                    help="summarize rocprofv3 CSV output of this command's timed iterations "
                         "instead (trace=, fetch=, write=, cfetch=, cwrite= directories)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="bytes of the copy-probe runs given to --summarize-profile")
    ap.add_argument("--write-traffic", action="store_true",
                    help="with --summarize-profile: write profiles/traffic.json")
    ap.add_argument("--fb-n", type=int, default=50000)
    ap.add_argument("--fb-k", type=int, default=256,
                    help="HD list length of the feedback and blob experiments (R_NX up to it)")
    ap.add_argument("--fb-perplexity", type=float, default=50.0,
                    help="perplexity of those experiments when --fb-k > 32")
    ap.add_argument("--fb-iters", type=int, default=2000)
    ap.add_argument("--fb-every", type=int, default=100)
    ap.add_argument("--dynamic", action="store_true",
                    help="run the online-use experiment (learned vs random placement) instead")
    ap.add_argument("--dyn-base", type=int, default=0, help="base points (0: 500,000)")
    ap.add_argument("--dyn-batches", type=int, default=10)
    ap.add_argument("--dyn-base-iters", type=int, default=2000)
    ap.add_argument("--dyn-cap", type=int, default=1000)
    ap.add_argument("--dyn-data", choices=("styles", "image"), default="styles",
                    help="styles: classes with a 3-dim style manifold; image: independent "
                         "pixel drops and jitter within a class")
    args = ap.parse_args()
    if args.summarize_phases:
        summarize_phases(args.summarize_phases)
        return
    if args.summarize_profile:
        summarize_profile(args)
        return
    if args.cpu_baseline_configs:
        print(json.dumps(cpu_baseline_configs(args)))
        return
    if args.copy_probe:
        import torch

        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path; the step would shard by point range.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from inputs.generators import f32_to_bf16_bits, make_workload, y_init, RUN_SEED
    from paper_2509_07681_amd import fsne as F

    if not os.path.exists(F.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.dynamic:
        print(json.dumps(dynamic_run(F, args)))
        return
    if args.mlp_train:
        print(json.dumps(mlp_train_run(F, args)))
        return
    if args.feedback:
        print(json.dumps(feedback_run(F, args)))
        return
    if args.hierarchy:
        print(json.dumps(hierarchy_run(F, args)))
        return
    if args.large:
        print(json.dumps(large_run(F, args)))
        return
    if args.scaling:
        print(json.dumps(scaling_run(F, args)))
        return
    if args.blobs_knn:
        print(json.dumps(blobs_knn_run(F, args)))
        return
    if args.memo_compare:
        print(json.dumps(memo_run(F, args)))
        return
    if args.image:
        print(json.dumps(image_run(F, args)))
        return
    X, _, cfg = make_workload("manifold_1m")
    N = X.shape[0]
    Y0 = y_init(N, cfg["d"])
    hp = F.fsne_default_hparams(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N / 12.0,
                                momentum=0.5, attr=12.0, n_neg=cfg["n_neg"], hd_mode=1)
    every, start = args.reorder_every, args.reorder_from
    W, K = args.warmup, args.steps
    renumbers = [t for t in range(W + K) if reorder_due(t, every, start)]

    def fresh(Xr, hpr):
        """A new embedding of the workload; with --reorder-data its points are
        first renumbered along a fixed projection of the data rows (set-up,
        before iteration 0, outside every timed region)."""
        e = F.Embedding(Xr, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hpr)
        orig = np.arange(N)
        if args.reorder_data:
            track_renumbering(orig, e.reorder_data())
        return e, orig

    # The timed region: iterations W .. W+K-1 of a fresh embedding, every
    # kernel launch bracketed by HIP events on the library's stream (read
    # after the region) for the per-kernel durations.
    emb, _ = fresh(X, hp)
    run_steps(emb, 0, W, every, start)
    emb.sync()
    emb.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(emb, W, K, every, start)
    emb.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / K
    kt = emb.kernel_times()
    emb.profile(False)
    st = emb.stats()
    assert st["nonfinite"] == 0, "embedding diverged"
    emb.close()

    # The same iterations again (the run is deterministic), one at a time, for
    # the candidate rows each of them loaded.
    emb, _ = fresh(X, hp)
    run_steps(emb, 0, W, every, start)
    _, hd_cand, ld_cand = profiled_steps(emb, W, K, every, start, N)
    emb.close()

    bpp = bytes_per_point(cfg, 4, hd_cand, ld_cand)
    sbpp = all_slot_bytes_per_point(cfg, 4)
    kernels = {}
    for k, (ms, n) in kt.items():
        avg = ms / max(n, 1)
        e = {"avg_ms": round(avg, 4), "launches": n}
        if k in bpp:
            gb = bpp[k] * N / 1e9
            e.update(algorithmic_GB=round(gb, 3), GBps=round(gb / (avg * 1e-3), 1),
                     frac=round(gb / (avg * 1e-3) / PEAK_HBM_GBS, 4),
                     all_slots_GB=round(sbpp[k] * N / 1e9, 3))
        kernels[k] = e
    kernels["hd_refine"]["candidate_rows_per_point"] = round(hd_cand, 3)
    kernels["ld_grad"]["candidate_rows_per_point"] = round(ld_cand, 3)
    ld_only_ms = sum(kernels[k]["avg_ms"] for k in ("ld_grad", "reduce", "update"))
    # the dominant kernel: of those with algorithmic bytes, the one that takes
    # longest per step in the timed iterations
    dom_name = max((k for k in kernels if "algorithmic_GB" in kernels[k]),
                   key=lambda k: kernels[k]["avg_ms"])
    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "manifold_1m: N=1,000,000 points on 50 seeded 8-dim linear "
                               "manifolds in R^128 (FP32 rows), d=16, K_hd=K_ld=32, 16 negatives, "
                               "alpha=1, perplexity 10; every timed step refines the HD lists"
                               + ("; before iteration 0 the points are renumbered along the "
                                  "Morton order of a fixed 3-axis projection of the data rows "
                                  "(set-up, untimed)" if args.reorder_data else "")
                               + (f"; the points are renumbered along the embedding's Morton "
                                  f"order every {every} iterations from iteration {start} on, "
                                  f"inside the timed region" if every > 0 else ""),
                   "N": N, "D": cfg["D"], "d": cfg["d"], "K_hd": cfg["K_hd"],
                   "K_ld": cfg["K_ld"], "n_neg": cfg["n_neg"], "hd_mode": "always",
                   "timed_iterations": [W, W + K - 1],
                   "reorder_data_at_setup": bool(args.reorder_data),
                   "renumbered_before_iterations": renumbers},
        "roofline": roofline(kernels, dom_name, W, K, [every, start, int(args.reorder_data)]),
        "kernels": kernels,
        "ld_only_ms_per_step": round(ld_only_ms, 4),
        "ld_only_iters_per_s": round(1000.0 / ld_only_ms, 2),
    }
    if renumbers or args.reorder_data:
        # the same iterations without any renumbering, for comparison
        emb = F.Embedding(X, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hp)
        emb.step(W)
        emb.sync()
        t0 = time.perf_counter()
        emb.step(K)
        emb.sync()
        ms_plain = (time.perf_counter() - t0) * 1e3 / K
        emb.close()
        out["no_reorder"] = {"ms_per_step": round(ms_plain, 4),
                             "iters_per_s": round(1000.0 / ms_plain, 3)}

    # the BF16 forms over the same iterations (at most 50 of them)
    Xb = f32_to_bf16_bits(X)
    forms = {}
    nf = min(K, 50)
    for name, dm in (("bf16_rows_direct", 0), ("bf16_mfma_screen", 1)):
        hpf = F.fsne_default_hparams(**{**hp.as_dict(), "dist_mode": dm})
        e2, orig = fresh(Xb, hpf)
        run_steps(e2, 0, W, every, start, orig)
        e2.sync()
        t2 = time.perf_counter()
        run_steps(e2, W, nf, every, start, orig)
        e2.sync()
        ms2 = (time.perf_counter() - t2) * 1e3 / nf
        kt2, _, _ = profiled_steps(e2, W + nf, min(nf, 10), every, start, N, orig)
        forms[name] = {"ms_per_step": round(ms2, 4), "iters_per_s": round(1000.0 / ms2, 2),
                       "hd_refine_ms": round(kt2["hd_refine"][0] / max(kt2["hd_refine"][1], 1),
                                             4)}
        if dm == 1:
            forms["bf16_error"] = bf16_error_statement(F, X[orig], Xb[orig], e2, cfg)
        e2.close()
    out["forms"] = forms
    progress(f"headline {out['value']} it/s and BF16 forms done")

    if not args.no_quality:
        from inputs.knn_metrics import exact_knn

        rng = np.random.default_rng(7)
        queries = rng.choice(N, args.queries, replace=False)
        _, ex_d2 = exact_knn(X, queries, cfg["K_hd"])
        qre = 100 if every > 0 else 0     # renumbering cadence under the coin
        rd = bool(args.reorder_data)
        runs = {"f32": quality_run(F, X, cfg, Y0, args.quality_iters, RUN_SEED, queries, ex_d2,
                                   reorder_every=qre, reorder_data=rd)}
        _, ex_b = exact_knn(Xb, queries, cfg["K_hd"])
        runs["bf16_rows_direct"] = quality_run(F, Xb, cfg, Y0, args.quality_iters, RUN_SEED,
                                               queries, ex_b, reorder_every=qre, reorder_data=rd)
        runs["bf16_mfma_screen"] = quality_run(F, Xb, cfg, Y0, args.quality_iters, RUN_SEED,
                                               queries, ex_b, dist_mode=1, reorder_every=qre,
                                               reorder_data=rd)
        # seconds for each form to reach 0.95 of the FP32 form's final recall
        target = round(0.95 * runs["f32"]["recall_at_32"], 4)
        for r in runs.values():
            r["seconds_to_target"] = seconds_to(r["curve"], target)
        # the FP32 run against HBM: algorithmic bytes of every launch of the
        # run (candidate rows per point as in the profiled steps) over its time
        r = runs["f32"]
        gb = (r["hd_refinements"] * bpp["hd_refine"]
              + r["iters"] * (bpp["ld_grad"] + bpp["update"])) * N / 1e9
        r["roofline"] = {"algorithmic_GB": round(gb, 1),
                         "GBps": round(gb / r["seconds"], 1),
                         "frac": round(gb / r["seconds"] / PEAK_HBM_GBS, 4),
                         "basis": "hd_refine bytes x refining iterations + (ld_grad + update) "
                                  "bytes x iterations, candidate rows per point from the "
                                  "profiled steps"}
        out["runs"] = runs
        out["runs_recall_target"] = target
    if not args.no_quality:
        progress("1000-iteration runs done")
    if not args.no_dynamic:
        out["dynamic"] = dynamic_run(F, args)
        progress("online-use experiment (styled generator) done")
        # the same experiment on the image-like generator itself (independent
        # pixel drops and jitter within a class: no low-dimensional structure
        # within a class, so the LD recall target is a far weaker signal)
        out["dynamic_image_generator"] = dynamic_run(F, argparse.Namespace(
            **{**vars(args), "dyn_data": "image"}))
    if not args.no_cpu_baseline:
        progress("online-use experiment (image-like generator) done" if not args.no_dynamic
                 else "starting the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(X, cfg, Y0, RUN_SEED)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
