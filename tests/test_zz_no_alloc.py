"""The allocation-free drift entry point against fsne_drift_points.

Two contexts hold the same state; one drifts points through
fsne_drift_points (staging allocated per call), the other through
fsne_drift_points_noalloc (staging in the library's fixed device array),
both called through the C ABI.  Two calls in a row, the second with fewer
points (the array keeps the first call's contents), then a step: every
state array must be identical.  A batch beyond the array's size is
rejected with FSNE_EINVAL and leaves the state untouched.
"""
import ctypes as C

import numpy as np
import pytest

from inputs.generators import f32_to_bf16_bits, image_like, manifolds, y_init

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

FIELDS = ["Y", "V", "hd_idx", "hd_d2", "ld_idx", "rec", "P", "flags"]

CASES = {
    # d = 5 (rows padded to 8), FP32 rows of 24
    "manifold_f32": (lambda: manifolds(n_manifolds=6, per_manifold=300, D=24, k=3, seed=61)[0],
                     5, 16, 8),
    # BF16 rows of 784 (the image-like workload's width), d = 2
    "image_bf16": (lambda: f32_to_bf16_bits(image_like(n_per_class=150, seed=62)[0]), 2, 32, 16),
}


def _pair(F, X, d, Kh, Kl):
    N = X.shape[0]
    hp = F.fsne_default_hparams(perplexity=6.0, lr=N / 12.0, n_neg=6, hd_mode=1)
    a = F.Embedding(X, y_init(N, d), d, Kh, Kl, seed=5, hp=hp, capacity=N)
    a.step(8)
    b = F.Embedding(X, y_init(N, d), d, Kh, Kl, seed=5, hp=hp, capacity=N)
    b.set_state(a.state())
    return a, b


def _same(a, b):
    ga, gb = a.state(FIELDS), b.state(FIELDS)
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), k


@pytest.mark.parametrize("name", list(CASES))
def test_noalloc_drift_matches_drift(fsne_lib, name):
    F = fsne_lib
    make, d, Kh, Kl = CASES[name]
    X = make()
    N = X.shape[0]
    a, b = _pair(F, X, d, Kh, Kl)
    L = F.load_library()
    rng = np.random.default_rng(3)
    for n in (400, 37):                      # the second call smaller than the first
        ids = np.sort(rng.choice(N, n, replace=False)).astype(np.int64)
        Xn = X[rng.permutation(N)[:n]].copy()
        Yn = rng.normal(size=(n, d)).astype(np.float32)
        print(f"{name}: drift of {n} points", flush=True)
        F.fsne_drift_points(a.ctx, ids, Xn, Yn)
        st = L.fsne_drift_points_noalloc(b.ctx, ids.ctypes.data_as(C.c_void_p),
                                         Xn.ctypes.data_as(C.c_void_p), n,
                                         Yn.ctypes.data_as(C.c_void_p))
        assert st == F.FSNE_OK, L.fsne_last_error(b.ctx)
        _same(a, b)
    # keep y (Yinit NULL)
    ids = np.arange(5, N, N // 50, dtype=np.int64)
    Xn = X[ids[::-1]].copy()
    F.fsne_drift_points(a.ctx, ids, Xn)
    F.fsne_drift_points_noalloc(b.ctx, ids, Xn)
    _same(a, b)
    a.step(3)
    b.step(3)
    _same(a, b)
    a.close()
    b.close()


def test_noalloc_drift_rejects_what_it_cannot_hold(fsne_lib):
    F = fsne_lib
    X = manifolds(n_manifolds=4, per_manifold=2000, D=1024, k=3, seed=63)[0]   # 4 KiB rows
    N, d = X.shape[0], 2
    hp = F.fsne_default_hparams(perplexity=6.0, lr=N / 12.0, n_neg=6, hd_mode=1)
    emb = F.Embedding(X, y_init(N, d), d, 16, 8, seed=5, hp=hp, capacity=N)
    before = emb.state(FIELDS)
    ids = np.arange(0, 5000, dtype=np.int64)     # 5000 x 4 KiB > 16 MiB
    with pytest.raises(F.FsneError) as e:
        F.fsne_drift_points_noalloc(emb.ctx, ids, X[:5000])
    assert e.value.status == F.FSNE_EINVAL and "scratch" in str(e.value)
    with pytest.raises(F.FsneError) as e:
        F.fsne_drift_points_noalloc(emb.ctx, np.array([4, 3], np.int64), X[:2])
    assert e.value.status == F.FSNE_EINVAL
    after = emb.state(FIELDS)
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    # the largest batch that fits goes through
    F.fsne_drift_points_noalloc(emb.ctx, np.arange(0, 3000, dtype=np.int64), X[N - 3000:])
    assert emb.stats()["nonfinite"] == 0
    emb.close()
