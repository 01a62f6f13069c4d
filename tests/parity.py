"""Comparison rules between the HIP library and the FP64 oracle.

Index lists: bit-exact, except where the two sides order two entries whose
exact (FP64) squared distances lie within the tie tolerance.  The tolerance
follows from the FP32 arithmetic of the HD distance on the GPU: each lane sums
n = VEC * chunks squared differences in order, then a G-lane butterfly adds
log2(G) levels, so |fl(d2) - d2| <= (n + log2 G + 2) u d2 with u = 2^-24, and
two entries can swap when their relative gap is below twice that bound.  The
tolerance is never below 1e-6 relative.

Floating-point results: gradients and partials within 1e-4 relative L2.
"""
from __future__ import annotations

import math

import numpy as np

U = 2.0 ** -24


def hd_geometry(D: int, bf16: bool):
    vec = (8 if D % 8 == 0 else 1) if bf16 else (4 if D % 4 == 0 else 1)
    V = -(-D // vec)
    G = 16 if V <= 16 else (32 if V <= 32 else 64)
    chunks = -(-V // G)
    return vec, G, chunks


def hd_tie_tol(D: int, bf16: bool = False) -> float:
    vec, G, chunks = hd_geometry(D, bf16)
    gamma = (vec * chunks + math.log2(G) + 2) * U
    return max(1e-6, 2.0 * gamma)


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def exact_d2(X, i, ids):
    """FP64 squared distances from row i to rows ids of X (float32 or bf16 bits)."""
    from inputs.generators import bf16_bits_to_f32

    Xf = bf16_bits_to_f32(X) if X.dtype == np.uint16 else X
    xi = Xf[i].astype(np.float64)
    return ((Xf[np.asarray(ids)].astype(np.float64) - xi) ** 2).sum(1)


def compare_hd_rows(X, gpu_idx, ora_idx, ora_d2, tol, rows=None):
    """Rows equal, or differing only at positions whose exact distances tie.

    Returns (number of rows that differ, number of rows that differ beyond the
    tie rule, list of offending rows).
    """
    N = gpu_idx.shape[0]
    rows = range(N) if rows is None else rows
    differ, bad = 0, []
    for i in rows:
        g, o = gpu_idx[i], ora_idx[i]
        if np.array_equal(g, o):
            continue
        differ += 1
        dg = exact_d2(X, i, g)
        # the GPU row must be a valid sorted list whose exact distances match the
        # oracle's at each position up to the tie tolerance
        if len(set(g.tolist())) != len(g) or i in set(g.tolist()):
            bad.append(i)
            continue
        if not np.all(np.abs(dg - ora_d2[i]) <= tol * np.maximum(ora_d2[i], 1e-30)):
            bad.append(i)
    return differ, len(bad), bad
