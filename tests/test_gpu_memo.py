"""Remembered rejections of the HD refinement change no result.

While X and the HD lists change only by refinement, a point's K-th HD
distance never grows (a merge keeps the K smallest keys of the old list and
the candidates), so a candidate that lost a merge would lose every later one.
The library skips such candidates (hparams.reject_memo = 1).  With the memory
on and off every state array must agree bit for bit, through insertion and
through the events that void the memory (drift, delete, a state load of the
lists, a change of the BF16 screen or of the HD metric), while fewer
candidate rows are read.
"""
import numpy as np
import pytest

from inputs.generators import f32_to_bf16_bits, image_like, manifolds, y_init, zipf_mixture

pytestmark = [pytest.mark.gpu]

FIELDS = ["Y", "V", "hd_idx", "hd_d2", "ld_idx", "rec", "P", "flags"]

# name: (rows, d, K_hd, K_ld, dist_mode); 3000 rows start, 100 are inserted later.
# Rows of 512 bytes or more remember 64 rejections with direct distances, others 32.
CASES = {
    # two points per wave, FP32 rows of 512 bytes (64 remembered)
    "manifold_3000_f32": (lambda: manifolds(per_manifold=62, seed=1003)[0], 16, 32, 32, 0),
    # one point per wave (K_hd = 64), BF16 rows of 512 bytes (64 remembered)
    "zipf_3000_bf16_k64": (lambda: f32_to_bf16_bits(
        zipf_mixture(N=3100, n_clusters=25, seed=1005)[0]), 32, 64, 32, 0),
    # one point per wave, BF16 rows of 256 bytes (32 remembered)
    "zipf_3000_bf16_d128_k64": (lambda: f32_to_bf16_bits(
        zipf_mixture(N=3100, D=128, n_clusters=25, seed=1009)[0]), 16, 64, 32, 0),
    # two points per wave, BF16 rows, matrix-core screen
    "manifold_3000_bf16_screen": (lambda: f32_to_bf16_bits(
        manifolds(per_manifold=62, seed=1007)[0]), 16, 32, 32, 1),
    # one point per wave over four row chunks, FP32 rows of 3136 bytes (64 remembered)
    "image_3000_f32_d784": (lambda: image_like(n_per_class=310, seed=1011)[0], 2, 32, 32, 0),
    # one point per wave over four row chunks with the matrix-core screen, K_hd = 64
    # (BF16 rows of 2048 bytes: 32 remembered under the screen, 64 after the switch)
    "zipf_3000_bf16_d1024_screen_k64": (lambda: f32_to_bf16_bits(
        zipf_mixture(N=3100, D=1024, n_clusters=25, seed=1013)[0]), 16, 64, 32, 1),
}


def _same(on, off, where):
    a, b = on.state(FIELDS), off.state(FIELDS)
    for k in FIELDS:
        x, y = a[k], b[k]
        if k == "flags":            # bit 0: list changed; bits 1..6 count rows read
            x, y = x & 1, y & 1
        assert np.array_equal(x, y), (where, k)
    sa, sb = on.stats(), off.stats()
    for k in ("N", "t", "E", "n_new", "Z", "last_fired", "nonfinite", "hd_refinements"):
        assert sa[k] == sb[k], (where, k, sa[k], sb[k])
    assert sa["nonfinite"] == 0
    # the same lists and draws give the same candidates; the memory only drops some
    assert sa["hd_cand_rows"] <= sb["hd_cand_rows"], where
    return sa["hd_cand_rows"], sb["hd_cand_rows"]


@pytest.mark.parametrize("case", list(CASES))
def test_memo_changes_no_result(fsne_lib, case):
    F = fsne_lib
    make, d, Kh, Kl, dist_mode = CASES[case]
    X_all = make()
    N = 3000
    X, X_new = X_all[:N], X_all[N:N + 100]
    base = dict(alpha=1.0, perplexity=10.0, lr=N / 12.0, n_neg=16, hd_mode=1,
                dist_mode=dist_mode, attr=12.0)
    embs = [F.Embedding(X, y_init(N, d), d, Kh, Kl, seed=11,
                        hp=F.fsne_default_hparams(**base, reject_memo=m), capacity=N + 100)
            for m in (1, 0)]
    on, off = embs
    assert on.hyperparams().reject_memo == 1 and off.hyperparams().reject_memo == 0

    def both(fn):
        for e in embs:
            fn(e)

    both(lambda e: e.step(40))
    r_on, r_off = _same(on, off, "40 steps")
    assert r_on < r_off, (r_on, r_off)      # repeated rejections were skipped
    both(lambda e: e.insert(X_new))
    both(lambda e: e.step(15))
    _same(on, off, "insert")
    ids = np.arange(0, 100, 2, dtype=np.int64)
    both(lambda e: e.drift(ids, X_all[ids + 500]))
    both(lambda e: e.step(15))
    _same(on, off, "drift")
    both(lambda e: e.delete(np.arange(7, 3100, 40, dtype=np.int64)))
    both(lambda e: e.step(15))
    _same(on, off, "delete")
    snap = on.state(["hd_idx", "hd_d2", "rec"])
    both(lambda e: e.set_state(snap))
    both(lambda e: e.step(10))
    _same(on, off, "state load")
    if X.dtype == np.uint16 and X.shape[1] % 16 == 0:
        both(lambda e: e.set_hyperparams(F.fsne_default_hparams(
            **{**e.hyperparams().as_dict(), "dist_mode": 1 - dist_mode})))
        both(lambda e: e.step(10))
        _same(on, off, "screen switch")
    if on.hyperparams().dist_mode == 0:
        # the angular metric: a switch clears the memory; drift recomputes the unit rows
        both(lambda e: e.set_hyperparams(F.fsne_default_hparams(
            **{**e.hyperparams().as_dict(), "metric": 1})))
        both(lambda e: e.step(15))
        _same(on, off, "angular metric")
        ids2 = np.arange(1, 60, 3, dtype=np.int64)
        both(lambda e: e.drift(ids2, X_all[ids2 + 700]))
        both(lambda e: e.step(10))
        _same(on, off, "angular drift")
    both(lambda e: e.set_hyperparams(F.fsne_default_hparams(
        **{**e.hyperparams().as_dict(), "hd_mode": 0, "attr": 1.0, "momentum": 0.8})))
    both(lambda e: e.step(30))
    _same(on, off, "coin")
    both(lambda e: e.close())
