"""Renumbering of the points (fsne_renumber, fsne_reorder).

A renumbering relabels the state: every per-point row moves to its new id
and every list entry is mapped, bit for bit; from the renumbered state the
method goes on exactly as the oracle does from its renumbered state.  The
Morton order of the embedding gives nearby ids to neighbours."""
import numpy as np
import pytest

from inputs.generators import blobs, f32_to_bf16_bits, manifolds, y_init
from tests.parity import check_injected_step, compare_hd_rows, hd_tie_tol, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

ROWS = ["Y", "V", "A", "R", "Zh", "rec", "P", "flags", "hd_d2"]


def _relabelled(s0, p, s1):
    for k in ROWS:
        assert np.array_equal(s1[k][p], s0[k]), k
    assert np.array_equal(s1["hd_idx"][p], p[s0["hd_idx"]])
    assert np.array_equal(s1["ld_idx"][p], p[s0["ld_idx"]])
    assert s1["E"] == s0["E"] and s1["t"] == s0["t"]


@pytest.mark.parametrize("bf16", [False, True])
def test_renumber_moves_every_row(fsne_lib, bf16):
    F = fsne_lib
    X, _ = blobs(n_clusters=8, per_cluster=250, D=32, seed=41)
    if bf16:
        X = f32_to_bf16_bits(X)
    N = X.shape[0]
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N / 12.0, n_neg=8, hd_mode=1, attr=12.0)
    emb = F.Embedding(X, y_init(N, 4), 4, 32, 16, seed=3, hp=hp)
    emb.step(20)
    s0 = emb.state()
    with pytest.raises(F.FsneError) as e:
        emb.renumber(np.zeros(N, dtype=np.int32))
    assert e.value.status == F.FSNE_EINVAL
    _relabelled(s0, np.arange(N), emb.state())
    p = np.random.default_rng(5).permutation(N).astype(np.int32)
    emb.renumber(p)
    _relabelled(s0, p, emb.state())
    # the rows of X moved too: the stored distances are those of the new ids
    emb.step(3)
    g = emb.state()
    Xf = X.astype(np.float32) if not bf16 else None
    if Xf is not None:
        Xp = np.empty_like(Xf)
        Xp[p] = Xf
        for i in range(0, N, 97):
            ex = ((Xp[g["hd_idx"][i]].astype(np.float64) - Xp[i]) ** 2).sum(1)
            np.testing.assert_allclose(g["hd_d2"][i], ex, rtol=1e-5)
    assert emb.stats()["nonfinite"] == 0
    emb.close()


def test_renumbered_steps_match_oracle(oracle_lib, fsne_lib):
    O, F = oracle_lib, fsne_lib
    X, _ = blobs(n_clusters=10, per_cluster=200, D=24, seed=43)
    N = X.shape[0]
    kw = dict(alpha=1.0, perplexity=10.0, lr=float(np.float32(N / 12.0)), momentum=0.5,
              attr=12.0, rep=1.0, n_neg=8, hd_mode=1, e_smooth=0.1, p_min=0.05)
    hp_o, hp_g = O.Hyper(**kw), F.fsne_default_hparams(**kw)
    Y0 = y_init(N, 2)
    S = O.OracleState(X, 2, 32, 16, 42, Y0).init(hp_o)
    emb = F.Embedding(X, Y0, 2, 32, 16, seed=42, hp=hp_g)
    for _ in range(3):
        S.step(hp_o)
    emb.set_state(S.round_to_f32().as_gpu_state())
    p = np.random.default_rng(6).permutation(N).astype(np.int32)
    S.renumber(p)
    emb.renumber(p)
    tol = hd_tie_tol(X.shape[1])

    def check_hd(g, S):
        differ, nbad, bad = compare_hd_rows(S.live("X"), g["hd_idx"], S.live("hd_idx"),
                                            S.live("hd_d2"), tol)
        assert nbad == 0, bad[:5]
        return np.all(g["hd_idx"] == S.live("hd_idx"), axis=1)

    # the first step from the GPU's own renumbered state, then from injected ones
    for it in range(3):
        check_injected_step(O, S, emb, hp_o, check_hd, inject=it > 0)
    emb.close()


def _locality(hd):
    N = hd.shape[0]
    return float(np.mean(np.abs(hd - np.arange(N)[:, None]))) / N


def test_reorder_gives_neighbours_nearby_ids(fsne_lib):
    F = fsne_lib
    X = manifolds(n_manifolds=20, per_manifold=400, seed=1003)[0]
    N = X.shape[0]
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N / 12.0, n_neg=16, hd_mode=1, attr=12.0)
    emb = F.Embedding(X, y_init(N, 16), 16, 32, 32, seed=3, hp=hp)
    emb.step(150)
    s0 = emb.state()
    before = _locality(s0["hd_idx"])
    p = emb.reorder()
    assert np.array_equal(np.sort(p), np.arange(N))
    _relabelled(s0, p, emb.state())
    after = _locality(emb.state()["hd_idx"])
    assert after < 0.3 * before, (before, after)
    # the run goes on from the renumbered state and the ids stay local
    emb.step(50)
    g = emb.state()
    assert emb.stats()["nonfinite"] == 0
    assert np.all(np.diff(g["hd_d2"], axis=1) >= 0)
    assert _locality(g["hd_idx"]) < 0.5 * before
    emb.close()


@pytest.mark.parametrize("N,d", [(7, 2), (1001, 2), (999, 3), (1234, 1)])
def test_reorder_low_dimensions_and_small_sizes(fsne_lib, N, d):
    """d <= 3 keys the Morton curve on the coordinates themselves; tiny and
    ragged sizes give valid permutations and relabelled states."""
    F = fsne_lib
    X = np.random.default_rng(N).normal(size=(N, 12)).astype(np.float32)
    Kh, Kl = min(5, N - 1), min(4, N - 1)
    hp = F.fsne_default_hparams(perplexity=min(3.0, Kh - 0.5), lr=max(N / 12.0, 1.0), n_neg=4,
                                hd_mode=1)
    emb = F.Embedding(X, y_init(N, d), d, Kh, Kl, seed=9, hp=hp)
    emb.step(30)
    s0 = emb.state()
    p = emb.reorder()
    assert np.array_equal(np.sort(p), np.arange(N))
    _relabelled(s0, p, emb.state())
    # the new order follows the Morton keys: ids grow along the first axis
    # within runs, so consecutive ids are close in the embedding
    Y = emb.Y()
    step = np.sqrt(((Y[1:] - Y[:-1]) ** 2).sum(1)).mean()
    rnd = np.sqrt(((Y[np.random.default_rng(1).permutation(N)][1:] - Y[:-1]) ** 2).sum(1)).mean()
    assert N < 100 or step < 0.5 * rnd, (step, rnd)
    emb.step(5)
    assert emb.stats()["nonfinite"] == 0
    emb.close()


def test_renumber_under_the_angular_metric(fsne_lib):
    """The unit rows move with X: after a renumbering every stored distance
    is the angular distance between the new ids' rows."""
    F = fsne_lib
    X, _ = blobs(n_clusters=6, per_cluster=200, D=20, seed=47)
    X = (X * np.exp2(np.random.default_rng(3).integers(-3, 4, size=(X.shape[0], 1)))).astype(
        np.float32)
    N = X.shape[0]
    hp = F.fsne_default_hparams(perplexity=8.0, lr=N / 12.0, n_neg=8, hd_mode=1, metric=1)
    emb = F.Embedding(X, y_init(N, 2), 2, 16, 8, seed=3, hp=hp)
    emb.step(10)
    p = emb.reorder()
    emb.step(3)
    g = emb.state()
    Xp = np.empty_like(X)
    Xp[p] = X
    U = Xp.astype(np.float64) / np.linalg.norm(Xp.astype(np.float64), axis=1, keepdims=True)
    for i in range(0, N, 37):
        ex = ((U[g["hd_idx"][i]] - U[i]) ** 2).sum(1)
        assert np.all(np.abs(g["hd_d2"][i] - ex) <= 1e-4 * np.sqrt(ex) + 1e-6 * ex + 1e-7), i
    emb.close()


def _spread(v, axes):
    if axes == 1:
        return v
    r = np.zeros_like(v)
    for b in range(30 // axes):
        r |= ((v >> b) & 1) << (b * axes)
    return r


def _morton_keys(Y):
    """The Morton keys of the renumbering, on the host in single precision:
    projection onto min(d, 3) axes (coordinates c = a, a+3, ... summed with
    alternating signs when d > 3), each axis scaled to its range and cut to
    30 / axes bits, bits interleaved."""
    N, d = Y.shape
    axes = min(d, 3)
    bits = 30 // axes
    top = np.float32((1 << bits) - 1)
    key = np.zeros(N, np.uint64)
    for a in range(axes):
        if d <= 3:
            v = Y[:, a].astype(np.float32)
        else:
            v = np.zeros(N, np.float32)
            for k, c in enumerate(range(a, d, 3)):
                v = (v - Y[:, c]) if k & 1 else (v + Y[:, c])
        lo, hi = v.min(), v.max()
        t = (v - lo) / (hi - lo) if hi > lo else np.zeros(N, np.float32)
        q = np.minimum(np.maximum(t * top, np.float32(0)), top).astype(np.uint64)
        key |= _spread(q, axes) << np.uint64(a)
    return key


@pytest.mark.parametrize("N,d", [(5000, 2), (70001, 3), (4097, 1), (12345, 16), (300, 5)])
def test_reorder_is_a_stable_sort_of_the_morton_keys(fsne_lib, N, d):
    """The new ids list the points by Morton key, equal keys in the order of
    the current ids (the library's own radix sort, several tiles and a
    ragged last one)."""
    F = fsne_lib
    X = manifolds(n_manifolds=10, per_manifold=-(-N // 10), D=24, k=3, seed=N)[0][:N]
    hp = F.fsne_default_hparams(perplexity=5.0, lr=max(N / 12.0, 1.0), n_neg=4, hd_mode=1)
    emb = F.Embedding(X, y_init(N, d), d, 8, 6, seed=9, hp=hp)
    emb.step(20)
    Y = emb.Y()
    p = emb.reorder()
    assert np.array_equal(np.sort(p), np.arange(N))
    old_of_new = np.argsort(p)
    k = _morton_keys(Y)[old_of_new].astype(np.int64)
    assert np.all(np.diff(k) >= 0)
    ties = np.diff(k) == 0
    assert np.all(np.diff(old_of_new)[ties] > 0)
    assert len(np.unique(k)) > N // 4       # keys spread, not all tied
    emb.close()


@pytest.mark.parametrize("bf16", [False, True])
def test_reorder_data_follows_a_projection_of_the_rows(oracle_lib, fsne_lib, bf16):
    """fsne_reorder_data right after init: a permutation that relabels the
    state exactly, orders the points by the Morton keys of the fixed +-1
    projection of their rows (keys recomputed on the host in double; the
    GPU's single-precision sums may move a key across a cell boundary), and
    gives true neighbours nearby ids."""
    O, F = oracle_lib, fsne_lib
    X = manifolds(n_manifolds=20, per_manifold=1000, D=64, k=4, seed=71)[0]
    if bf16:
        X = f32_to_bf16_bits(X)
    N, D = X.shape
    hp = F.fsne_default_hparams(perplexity=8.0, lr=N / 12.0, n_neg=8, hd_mode=1)
    emb = F.Embedding(X, y_init(N, 2), 2, 16, 8, seed=7, hp=hp)
    s0 = emb.state()
    p = emb.reorder_data()
    assert np.array_equal(np.sort(p), np.arange(N))
    _relabelled(s0, p, emb.state())
    # host keys from the same signs (Philox block (k, a, 12, 0), bit 0)
    sign = np.array([[-1.0 if O.philox4x32_10([k, a, 12, 0], [7, 0])[0] & 1 else 1.0
                      for a in range(3)] for k in range(D)])
    from inputs.generators import bf16_bits_to_f32
    Xf = (bf16_bits_to_f32(X) if bf16 else X).astype(np.float64)
    proj = Xf @ sign
    keys = _morton_keys(proj.astype(np.float32))
    k = keys[np.argsort(p)].astype(np.int64)
    assert np.mean(np.diff(k) >= 0) > 0.99
    # neighbours in R^D are near in the new ids
    from inputs.knn_metrics import exact_knn
    q = np.random.default_rng(1).choice(N, 200, replace=False)
    nn, _ = exact_knn(X, q, 8)
    gap = np.abs(p[nn] - p[q][:, None])
    assert np.median(gap) < N / 50, np.median(gap)
    emb.step(5)
    assert emb.stats()["nonfinite"] == 0
    emb.close()
