"""Neighbour-list quality metrics for evaluation (not part of the method).

Exact K-NN ground truth by brute force on the CPU: candidates from the
expanded form in float32 (torch matmul), then their distances recomputed
directly in float64 so the order is exact.
"""
from __future__ import annotations

import numpy as np


def _as_f32(X):
    from inputs.generators import bf16_bits_to_f32

    return bf16_bits_to_f32(X) if X.dtype == np.uint16 else np.asarray(X, dtype=np.float32)


def exact_knn(X, queries, K, batch=256):
    """Exact K nearest neighbours (self excluded) of the query rows: (idx, d2 float64)."""
    import torch

    Xf = _as_f32(X)
    Xt = torch.from_numpy(Xf)
    nrm = (Xt * Xt).sum(1)
    q = np.asarray(queries, dtype=np.int64)
    out_i = np.empty((q.size, K), dtype=np.int64)
    out_d = np.empty((q.size, K), dtype=np.float64)
    extra = min(Xf.shape[0] - 1, 2 * K + 8)
    for s in range(0, q.size, batch):
        qq = q[s:s + batch]
        Q = Xt[qq]
        approx = nrm[qq][:, None] + nrm[None, :] - 2.0 * (Q @ Xt.T)
        approx[torch.arange(qq.size), torch.from_numpy(qq)] = float("inf")
        cand = torch.topk(approx, extra + 1, dim=1, largest=False).indices.numpy()
        for r, i in enumerate(qq):
            c = cand[r][cand[r] != i][:extra]
            d = ((Xf[c].astype(np.float64) - Xf[i].astype(np.float64)) ** 2).sum(1)
            order = np.lexsort((c, d))[:K]
            out_i[s + r] = c[order]
            out_d[s + r] = d[order]
    return out_i, out_d


def recall_at_k(lists, X, queries, exact_d2, rel_tie=1e-6):
    """Fraction of list entries whose exact distance is within the exact K-th
    distance (times 1 + rel_tie): a hit at a tie counts."""
    Xf = _as_f32(X)
    q = np.asarray(queries, dtype=np.int64)
    K = exact_d2.shape[1]
    hits = 0
    for r, i in enumerate(q):
        lst = np.asarray(lists[i][:K], dtype=np.int64)
        d = ((Xf[lst].astype(np.float64) - Xf[i].astype(np.float64)) ** 2).sum(1)
        hits += int(np.sum(d <= exact_d2[r, K - 1] * (1.0 + rel_tie)))
    return hits / (q.size * K)


def knn_on_device(Xd, queries, K, chunk=256, direct=False):
    """K nearest neighbours (self excluded) of rows ``queries`` among all rows
    of the float32 device tensor ``Xd``, by brute force on the device; for
    recall measurements at sizes where the CPU brute force is too slow.

    ``direct`` sums squared coordinate differences (use for low-dimensional
    embeddings far from the origin); otherwise the expanded form
    |q|^2 + |x|^2 - 2 q.x is used.  Returns an int64 numpy array (nq, K).
    """
    import torch

    q = torch.as_tensor(np.asarray(queries, dtype=np.int64), device=Xd.device)
    nrm = None if direct else (Xd * Xd).sum(1)
    out = []
    for s in range(0, q.numel(), chunk):
        qq = q[s:s + chunk]
        if direct:
            Q = Xd[qq]
            d = torch.zeros((qq.numel(), Xd.shape[0]), dtype=torch.float32, device=Xd.device)
            for c in range(Xd.shape[1]):
                d += (Xd[None, :, c] - Q[:, c, None]) ** 2
        else:
            d = nrm[qq][:, None] + nrm[None, :] - 2.0 * (Xd[qq] @ Xd.T)
        d[torch.arange(qq.numel(), device=Xd.device), qq] = float("inf")
        out.append(torch.topk(d, K, dim=1, largest=False).indices.cpu())
    return torch.cat(out).numpy()


def set_recall(a, b):
    """Mean over rows of |a_r ∩ b_r| / K for two (n, K) index arrays."""
    K = a.shape[1]
    return float(np.mean([len(set(x.tolist()) & set(y.tolist())) / K for x, y in zip(a, b)]))


def rnx_curve(est, exact, N):
    """R_NX(K) for K = 1 .. Kmax of estimated neighbour lists against exact ones.

    est, exact: (n, Kmax) index arrays, each row sorted nearest first (so its
    first K entries are that row's K-neighbourhood).  With Q_NX(K) the mean
    of |est_K ∩ exact_K| / K over the rows, R_NX(K) rescales it so that 0 is
    a random neighbourhood and 1 a perfect one:
        R_NX(K) = ((N - 1) Q_NX(K) - K) / (N - 1 - K)      (Lee and Verleysen)
    """
    est = np.asarray(est, dtype=np.int64)
    exact = np.asarray(exact, dtype=np.int64)
    n, Kmax = exact.shape
    hits = np.zeros(Kmax + 1, dtype=np.float64)
    for r in range(n):
        pos = {int(j): k for k, j in enumerate(exact[r])}
        # entry k of the estimate, at exact rank q, is shared by both
        # K-neighbourhoods for every K > max(k, q)
        for k, j in enumerate(est[r][:Kmax]):
            q = pos.get(int(j))
            if q is not None:
                hits[max(k, q) + 1] += 1.0
    shared = np.cumsum(hits)[1:]
    K = np.arange(1, Kmax + 1, dtype=np.float64)
    Q = shared / (n * K)
    return ((N - 1) * Q - K) / (N - 1 - K)


def rnx_points(est, exact, N):
    """Per-row R_NX(K), K = 1 .. Kmax: row r's |est_K ∩ exact_K| / K rescaled
    as in rnx_curve (whose value is the mean of these rows).  Returns an
    (n, Kmax) array."""
    est = np.asarray(est, dtype=np.int64)
    exact = np.asarray(exact, dtype=np.int64)
    n, Kmax = exact.shape
    hits = np.zeros((n, Kmax + 1), dtype=np.float64)
    for r in range(n):
        pos = {int(j): k for k, j in enumerate(exact[r])}
        for k, j in enumerate(est[r][:Kmax]):
            q = pos.get(int(j))
            if q is not None:
                hits[r, max(k, q) + 1] += 1.0
    shared = np.cumsum(hits, axis=1)[:, 1:]
    K = np.arange(1, Kmax + 1, dtype=np.float64)
    return ((N - 1) * shared / K - K) / (N - 1 - K)


def rnx_auc(curve):
    """Area under R_NX(K) on a log scale of K: sum R(K)/K over sum 1/K."""
    K = np.arange(1, len(curve) + 1, dtype=np.float64)
    return float(np.sum(np.asarray(curve) / K) / np.sum(1.0 / K))


def exact_knn_device(Xd, X_host, queries, K, chunk=128):
    """exact_knn for large sets: candidates (2K + 8 per query) from the
    expanded form on the device (float32 tensor Xd), then their distances
    recomputed in float64 on the host from X_host (float32 rows or bf16 bits)
    so the order is exact.  Returns (idx, d2 float64)."""
    q = np.asarray(queries, dtype=np.int64)
    cand = knn_on_device(Xd, q, min(Xd.shape[0] - 1, 2 * K + 8), chunk=chunk)
    out_i = np.empty((q.size, K), dtype=np.int64)
    out_d = np.empty((q.size, K), dtype=np.float64)
    for r, i in enumerate(q):
        c = cand[r]
        d = ((_as_f32(X_host[c]).astype(np.float64) -
              _as_f32(X_host[i:i + 1]).astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((c, d))[:K]
        out_i[r] = c[order]
        out_d[r] = d[order]
    return out_i, out_d
