#!/usr/bin/env python3
"""Benchmark of the FUnc-SNE step on one MI355X.

Workload: 1,000,000 points on 50 seeded 8-dim linear manifolds in R^128
(FP32 rows), embedded in d = 16 with K_hd = K_ld = 32, 16 negatives,
alpha = 1, perplexity 10.  A timed step is one full iteration with the HD
refinement on (every row of the step runs: coin, candidates, HD distances,
merge, recalibration, affinities, LD refinement, gradient, Z, update).

Prints one JSON line.  Besides the headline it reports the per-kernel
roofline of the dominant kernel (HD refinement), the other kernels, the
1000-iteration run of the workload under the refinement coin for the FP32
and the BF16 forms (wall seconds and HD recall@32 on a query sample), and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2509_07681_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_point(cfg, xbytes, hd_cand, ld_cand):
    """Bytes each kernel must move per point, no cache reuse assumed.

    hd_cand / ld_cand: mean number of distinct candidate rows per point that
    the kernels loaded (duplicate slots are dropped before any row is read).
    """
    D, d, Kh, Kl, nn = cfg["D"], cfg["d"], cfg["K_hd"], cfg["K_ld"], cfg["n_neg"]
    dp = 2
    while dp < d:
        dp *= 2
    sx, sy = D * xbytes, 4 * dp
    hd = sx * (1 + hd_cand) + 16 * Kh + 4 * Kl + 96 + 33
    ld = sy * (1 + Kl + ld_cand + Kh + nn + 2) + 8 * Kh + 8 * Kl + 96 + 5
    upd = 6 * sy
    return dict(hd_refine=hd, ld_grad=ld, update=upd)


def survey_bytes_per_point(cfg, xbytes):
    """The same with every one of the 32 candidate slots counted."""
    D, d, Kh, Kl, nn = cfg["D"], cfg["d"], cfg["K_hd"], cfg["K_ld"], cfg["n_neg"]
    sx, sy = D * xbytes, 4 * d
    hd = (C_SLOTS + 1) * sx + 96 + 16 * Kh + 12 + 24 * Kh + 12
    ld = sy + 8 * Kl + 8 * Kh + 96 + (Kl + C_SLOTS + Kh + nn) * sy + 2 * sy
    return dict(hd_refine=hd, ld_grad=ld, update=6 * sy)


def schedule(F, base, t):
    """Early exaggeration 12 with momentum 0.5 for 250 iterations, then 1 and 0.8."""
    early = t < 250
    return F.fsne_default_hparams(**{**base, "attr": 12.0 if early else 1.0,
                                     "momentum": 0.5 if early else 0.8})


def quality_run(F, X, cfg, Y0, n_iter, seed, queries, ex_d2, dist_mode=0):
    from inputs.knn_metrics import recall_at_k

    N = X.shape[0]
    base = dict(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N / 12.0,
                n_neg=cfg["n_neg"], hd_mode=0, dist_mode=dist_mode)
    emb = F.Embedding(X, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=seed,
                      hp=schedule(F, base, 0))
    emb.sync()
    t0 = time.perf_counter()
    done, fires = 0, 0
    while done < n_iter:
        n = min(250 - done, n_iter - done) if done < 250 else n_iter - done
        emb.set_hyperparams(schedule(F, base, done))
        emb.step(n)
        done += n
    emb.sync()
    secs = time.perf_counter() - t0
    st = emb.stats()
    idx, _ = emb.knn(0)
    rec = recall_at_k(idx, X, queries, ex_d2)
    emb.close()
    return dict(iters=n_iter, seconds=round(secs, 3), iters_per_s=round(n_iter / secs, 2),
                recall_at_32=round(rec, 4), final_E=round(float(st["E"]), 4),
                nonfinite=int(st["nonfinite"]))


def cpu_baseline(X, cfg, Y0, seed):
    from oracle import oracle as O

    N = X.shape[0]
    hp = O.Hyper(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=float(N / 12.0),
                 momentum=0.5, attr=12.0, n_neg=cfg["n_neg"], hd_mode=1)
    S = O.OracleState(X, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed, Y0).init(hp)
    t0 = time.perf_counter()
    S.step(hp)
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 4), "unit": "iters/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"1 iteration with the HD refinement on, over all N={N} points of the "
                      "same workload (FP64 C oracle, OpenMP over points), after an untimed "
                      f"oracle init; {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--quality-iters", type=int, default=1000)
    ap.add_argument("--queries", type=int, default=1000)
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device to device (counter calibration)")
    args = ap.parse_args()
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
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the step shards by point range; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from inputs.generators import f32_to_bf16_bits, make_workload, y_init, RUN_SEED
    from paper_2509_07681_amd import fsne as F

    if not os.path.exists(F.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    X, _, cfg = make_workload("manifold_1m")
    N = X.shape[0]
    Y0 = y_init(N, cfg["d"])
    hp = F.fsne_default_hparams(alpha=cfg["alpha"], perplexity=cfg["perplexity"], lr=N / 12.0,
                                momentum=0.5, attr=12.0, n_neg=cfg["n_neg"], hd_mode=1)
    emb = F.Embedding(X, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hp)
    emb.step(args.warmup)
    emb.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    emb.step(args.steps)
    emb.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    st = emb.stats()
    assert st["nonfinite"] == 0, "embedding diverged"

    # per-kernel durations from HIP events recorded on the library's stream,
    # and the candidate rows each iteration actually loaded
    n_prof = min(args.steps, 50)
    emb.profile(True)
    hd_c, ld_c = [], []
    for _ in range(n_prof):
        emb.step(1)
        s1 = emb.stats()
        hd_c.append(s1["hd_cand_rows"] / N)
        ld_c.append(s1["ld_cand_rows"] / N)
    kt = emb.kernel_times()
    emb.profile(False)
    emb.close()

    hd_cand, ld_cand = float(np.mean(hd_c)), float(np.mean(ld_c))
    bpp = bytes_per_point(cfg, 4, hd_cand, ld_cand)
    sbpp = survey_bytes_per_point(cfg, 4)
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
    dom = kernels["hd_refine"]
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("source_hash") == kernel_source_hash() and "hd_refine" in rec.get("per_launch_GB", {}):
            traffic = rec["per_launch_GB"]["hd_refine"]
    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms_step, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "manifold_1m: N=1,000,000 points on 50 seeded 8-dim linear "
                               "manifolds in R^128 (FP32 rows), d=16, K_hd=K_ld=32, 16 negatives, "
                               "alpha=1, perplexity 10; every timed step refines the HD lists",
                   "N": N, "D": cfg["D"], "d": cfg["d"], "K_hd": cfg["K_hd"],
                   "K_ld": cfg["K_ld"], "n_neg": cfg["n_neg"], "hd_mode": "always"},
        "roofline": {"bound": "hbm", "kernel": "hd_refine", "achieved": dom["GBps"],
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": dom["frac"],
                     "traffic": traffic, "traffic_unit": "GB per launch (FETCH_SIZE x2.0 "
                     "+ WRITE_SIZE x1.0, copy-calibrated)"},
        "kernels": kernels,
        "ld_only_ms_per_step": round(ld_only_ms, 4),
        "ld_only_iters_per_s": round(1000.0 / ld_only_ms, 2),
    }

    # the BF16 forms: step time with the HD refinement on
    Xb = f32_to_bf16_bits(X)
    forms = {}
    for name, dm in (("bf16_rows_direct", 0), ("bf16_mfma_screen", 1)):
        hpf = F.fsne_default_hparams(**{**hp.as_dict(), "dist_mode": dm})
        e2 = F.Embedding(Xb, Y0, cfg["d"], cfg["K_hd"], cfg["K_ld"], seed=RUN_SEED, hp=hpf)
        e2.step(args.warmup)
        e2.profile(True)
        nf = min(args.steps, 50)
        e2.step(nf)
        kt2 = e2.kernel_times()
        e2.sync()
        t2 = time.perf_counter()
        e2.step(nf)
        e2.sync()
        ms2 = (time.perf_counter() - t2) * 1e3 / nf
        e2.close()
        forms[name] = {"ms_per_step": round(ms2, 4), "iters_per_s": round(1000.0 / ms2, 2),
                       "hd_refine_ms": round(kt2["hd_refine"][0] / max(kt2["hd_refine"][1], 1), 4)}
    out["forms"] = forms

    if not args.no_quality:
        from inputs.knn_metrics import exact_knn

        rng = np.random.default_rng(7)
        queries = rng.choice(N, args.queries, replace=False)
        _, ex_d2 = exact_knn(X, queries, cfg["K_hd"])
        runs = {"f32": quality_run(F, X, cfg, Y0, args.quality_iters, RUN_SEED, queries, ex_d2)}
        _, ex_b = exact_knn(Xb, queries, cfg["K_hd"])
        runs["bf16_rows_direct"] = quality_run(F, Xb, cfg, Y0, args.quality_iters, RUN_SEED,
                                               queries, ex_b)
        runs["bf16_mfma_screen"] = quality_run(F, Xb, cfg, Y0, args.quality_iters, RUN_SEED,
                                               queries, ex_b, dist_mode=1)
        out["runs"] = runs
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, cfg, Y0, RUN_SEED)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
