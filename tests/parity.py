"""Comparison rules between the HIP library and the FP64 oracle.

Index lists: bit-exact, except where the two sides order two entries whose
exact (FP64) squared distances lie within the tie tolerance.  The tolerance
follows from the FP32 arithmetic of the HD distance on the GPU: each lane sums
n = VEC * chunks squared differences in order, then a G-lane butterfly adds
log2(G) levels, so |fl(d2) - d2| <= (n + log2 G + 2) u d2 with u = 2^-24, and
two entries can swap when their relative gap is below twice that bound.  The
tolerance is never below 1e-6 relative.

LD lists: the oracle decides membership with the exact (FP64) distance
|y_i - y_j|^2 of the same single-precision coordinates; the GPU takes it in
FP32: each difference and square rounded, the d squares summed as a pairwise
tree of log2(DP) levels (DP = d padded to a power of two), so
|fl(q) - q| <= (3 + log2 DP + 1) u q, and two entries can swap when their
relative gap is below twice that.  Rows equal, or differing only at such
positions.

Coin: the oracle fires when the 32-bit draw u < p 2^32 exactly; the GPU
compares with floor(fl(p) 2^32) in FP32, so the two can disagree only when
|u - p 2^32| is within the FP32 rounding of p 2^32, below 2^32 * 1e-6.

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
            if len(bad) <= 2:
                k = np.nonzero(g != o)[0]
                print(f"HD row {i} differs beyond the tie rule at positions {k[:8]}: "
                      f"gpu ids {g[k[:8]]} d2 {dg[k[:8]]}, oracle ids {o[k[:8]]} "
                      f"d2 {np.asarray(ora_d2[i])[k[:8]]}; gpu ids missing from the oracle "
                      f"row {sorted(set(g.tolist()) - set(o.tolist()))[:8]}, oracle ids "
                      f"missing from the gpu row {sorted(set(o.tolist()) - set(g.tolist()))[:8]}",
                      flush=True)
    return differ, len(bad), bad


def pad_dim(d: int) -> int:
    dp = 2
    while dp < d:
        dp *= 2
    return dp


def ld_tie_tol(d: int) -> float:
    gamma = (3 + math.log2(pad_dim(d)) + 1) * U
    return max(1e-6, 2.0 * gamma)


COIN_BAND = 2.0 ** 32 * 1e-6


def compare_ld_rows(Y, gpu_idx, ora_idx, tol, rows=None):
    """LD rows equal, or differing only where exact distances tie.

    Y: the single-precision coordinates both sides started from (as float64).
    Returns (mask of rows that are equal, number of rows that differ, rows
    that differ beyond the tie rule)."""
    N = gpu_idx.shape[0]
    rows = range(N) if rows is None else rows
    equal = np.all(gpu_idx == ora_idx, axis=1)
    differ, bad = 0, []
    for i in rows:
        if equal[i]:
            continue
        differ += 1
        g, o = gpu_idx[i], ora_idx[i]
        if len(set(g.tolist())) != len(g) or i in set(g.tolist()) or np.any(g < 0) \
                or np.any(g >= Y.shape[0]):
            bad.append(i)
            continue
        dg = ((Y[g] - Y[i]) ** 2).sum(1)
        do = ((Y[o] - Y[i]) ** 2).sum(1)
        if not np.all(np.abs(dg - do) <= tol * np.maximum(do, 1e-300)):
            bad.append(i)
    return equal, differ, bad


def check_injected_step(O, S, emb, hp_o, check_hd, fp_tol=1e-4, tie_rows=None, zh_tol=1e-5,
                        inject=True):
    """One iteration from the same state on both sides, compared in full.

    The oracle's state is rounded to single precision and injected into the
    GPU; both take one step.  Then:
    * coin (up to the FP32 band), t, E (up to the smoothing of a tie-row count);
    * every HD row by check_hd(g, S) -> mask of equal rows (tie rule inside);
    * the end of the HD phase phase-wise for EVERY point: the oracle
      recalibrates the GPU's new lists (its flags) and recomputes P from them;
      calibration and P must match the GPU's at fp_tol;
    * the LD phase phase-wise for EVERY point: the oracle's LD phase runs on
      the GPU's HD lists and P; LD rows by the LD tie rule, A over all points,
      R, Zh and the update over every point whose LD row is equal;
    * the whole oracle step on the points whose inputs agree exactly (HD row
      and its neighbours' rows equal).
    inject=False: the GPU already holds S (rounded to single precision).
    Returns (GPU state, oracle step output); S has advanced by one step."""
    N = S.N
    tie_rows = max(3, N // 500) if tie_rows is None else tie_rows
    S.round_to_f32()
    pre = S.copy()
    if inject:
        emb.set_state(S.as_gpu_state())
    Y0 = S.live("Y").copy()
    out = S.step(hp_o, want_partials=True)
    emb.step(1)
    st = emb.stats()
    g = emb.state()
    fired = st["last_fired"]
    if fired != out["fired"]:
        margin = O.coin_margin(pre.E[0], int(pre.t[0]), pre.seed, hp_o.p_min)
        assert abs(margin) <= COIN_BAND, (fired, out["fired"], margin)
        S.__dict__.update(pre.copy().__dict__)
        out = S.step(hp_o.copy(hd_mode=1 if fired else 2), want_partials=True)
    assert g["t"] == out["t"]
    # HD rows (every row)
    same = check_hd(g, S)
    differ = int((~same).sum())
    assert differ <= tie_rows, f"{differ} HD rows differ at ties"
    if fired:
        assert np.array_equal(g["flags"][same] & 1, S.live("flags")[same])
        assert abs(st["n_new"] - out["n_new"]) <= differ
    lam = hp_o.e_smooth
    assert abs(g["E"] - out["E"]) <= 2.0 ** -22 * out["E"] + lam * differ / N + 1e-12
    # the end of the HD phase from the GPU's lists, every point
    if fired:
        ph = pre.copy()
        ph.hd_idx[:N] = g["hd_idx"]
        ph.hd_d2[:N] = g["hd_d2"]
        ph.flags[:N] = g["flags"] & 1
        ph.hd_finish(hp_o)
        assert rel_l2(g["rec"][:, 0], ph.live("beta")) < fp_tol
        assert rel_l2(g["rec"][:, 3], ph.live("invS")) < fp_tol
        P_ref = ph.live("P")
    else:
        P_ref = pre.live("P")
        assert np.array_equal(g["hd_idx"], pre.live("hd_idx"))
    assert rel_l2(g["P"], P_ref) < fp_tol
    # the LD phase from the GPU's HD lists and P, every point
    ld_o, A_o, R_o, Zh_o = pre.ld_phase(hp_o, g["hd_idx"], g["P"].astype(np.float64))
    lt = ld_tie_tol(S.d)
    eq, ldiff, lbad = compare_ld_rows(Y0, g["ld_idx"], ld_o, lt)
    assert not lbad, f"LD rows beyond the tie rule: {lbad[:10]}"
    assert ldiff <= tie_rows, f"{ldiff} LD rows differ at ties"
    assert rel_l2(g["A"], A_o) < fp_tol
    assert rel_l2(g["R"][eq], R_o[eq]) < fp_tol
    assert np.all(np.abs(g["Zh"][eq] - Zh_o[eq]) <= zh_tol * Zh_o[eq])
    Z_o = Zh_o.sum()
    assert abs(st["Z"] - Z_o) <= fp_tol * Z_o
    dY_o = hp_o.momentum * pre.live("V") - hp_o.lr * 4.0 * (hp_o.attr * A_o - hp_o.rep * R_o / Z_o)
    dY_g = g["Y"].astype(np.float64) - Y0
    assert rel_l2(dY_g[eq], dY_o[eq]) < fp_tol
    # the whole oracle step where the inputs agree exactly
    hd = S.live("hd_idx")
    clean = same & np.all(same[hd], axis=1)
    if clean.any():
        assert rel_l2(g["P"][clean], S.live("P")[clean]) < fp_tol
        eq2, _, lbad2 = compare_ld_rows(Y0, g["ld_idx"], S.live("ld_idx"), lt,
                                        rows=np.where(clean)[0])
        assert not lbad2, lbad2[:10]
        ok = clean & eq2
        assert rel_l2(g["A"][ok], out["A"][ok]) < fp_tol
        assert rel_l2(g["R"][ok], out["R"][ok]) < fp_tol
        assert np.all(np.abs(g["Zh"][ok] - out["Zh"][ok]) <= zh_tol * out["Zh"][ok])
        assert rel_l2(dY_g[ok], (S.live("Y") - Y0)[ok]) < fp_tol
    return g, out
