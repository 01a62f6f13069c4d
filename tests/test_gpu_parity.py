"""GPU (HIP) vs FP64 oracle, element by element, with the oracle's state
injected before every compared iteration.

Sizes: a few thousand points (hundreds of 4-wave blocks) with ragged tails;
the full-size workloads are covered by test_gpu_fullsize.py.
"""
import numpy as np
import pytest

from inputs.generators import (blobs, f32_to_bf16_bits, image_like, manifolds, y_init,
                               zipf_mixture)
from tests.parity import check_injected_step, compare_hd_rows, hd_tie_tol, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def _f32(v):
    return float(np.float32(v))


def make_hp(O, F, N, **kw):
    """The same hyperparameters for both sides (the oracle gets the FP32 values)."""
    base = dict(alpha=1.0, perplexity=10.0, lr=N / 12.0, momentum=0.5, attr=12.0, rep=1.0,
                n_neg=8, hd_mode=0, e_smooth=0.1, p_min=0.05)
    base.update(kw)
    hp_o = O.Hyper(**{k: (_f32(v) if isinstance(v, float) else v) for k, v in base.items()})
    hp_g = F.fsne_default_hparams(**base)
    return hp_o, hp_g


WORKLOADS = {
    "blobs_2000": lambda: (blobs(seed=1001)[0], dict(d=2, K_hd=32, K_ld=16, n_neg=8, alpha=1.0,
                                                      perplexity=10.0)),
    "blobs_1237": lambda: (blobs(seed=1001)[0][:1237],
                           dict(d=2, K_hd=32, K_ld=16, n_neg=8, alpha=1.0, perplexity=10.0)),
    "image_3001_a05": lambda: (image_like(n_per_class=301, seed=1002)[0][:3001],
                               dict(d=2, K_hd=32, K_ld=32, n_neg=16, alpha=0.5, perplexity=10.0)),
    "image_2003_a4": lambda: (image_like(n_per_class=201, seed=1002)[0][:2003],
                              dict(d=2, K_hd=32, K_ld=32, n_neg=16, alpha=4.0, perplexity=10.0)),
    "manifold_4003_f32": lambda: (manifolds(per_manifold=81, seed=1003)[0][:4003],
                                  dict(d=16, K_hd=32, K_ld=32, n_neg=16, alpha=1.0,
                                       perplexity=10.0)),
    "manifold_4003_bf16": lambda: (f32_to_bf16_bits(manifolds(per_manifold=81, seed=1003)[0][:4003]),
                                   dict(d=16, K_hd=32, K_ld=32, n_neg=16, alpha=1.0,
                                        perplexity=10.0)),
    "zipf_3000_bf16": lambda: (f32_to_bf16_bits(zipf_mixture(N=3000, n_clusters=30, seed=1005)[0]),
                               dict(d=32, K_hd=64, K_ld=32, n_neg=32, alpha=0.5, perplexity=20.0)),
    # LD lists longer than one wave's candidate merge (K_ld > 32)
    "long_ld_1500": lambda: (manifolds(per_manifold=30, seed=1007)[0][:1500],
                             dict(d=8, K_hd=40, K_ld=48, n_neg=12, alpha=1.0, perplexity=12.0)),
    "wide_ld_1100_bf16": lambda: (f32_to_bf16_bits(zipf_mixture(N=1100, n_clusters=12,
                                                                seed=1008)[0]),
                                  dict(d=32, K_hd=48, K_ld=64, n_neg=24, alpha=0.5,
                                       perplexity=15.0)),
    # the largest sizes the library accepts: D at fsne_max_dim, d = K_hd = K_ld
    # = n_neg = 64 (low-noise 4-dim manifolds, so that neighbour distances are
    # well separated at this D)
    # At D = 4096 the tie tolerance is 4e-6 relative, so a few rows differ at
    # ties, and with K_hd = N / 5 each such row sits in ~64 other points'
    # lists; the phase-wise checks still cover every point.
    "max_f32_320": lambda: (manifolds(n_manifolds=5, per_manifold=64, D=4096, k=4,
                                      noise=0.005, seed=1009)[0],
                            dict(d=64, K_hd=64, K_ld=64, n_neg=64, alpha=1.0, perplexity=20.0,
                                 tie_rows=8)),
    "max_bf16_300": lambda: (f32_to_bf16_bits(manifolds(n_manifolds=5, per_manifold=60, D=2048,
                                                        k=4, noise=0.005, seed=1010)[0]),
                             dict(d=64, K_hd=64, K_ld=64, n_neg=64, alpha=0.7,
                                  perplexity=15.0, tie_rows=8)),
    # D with no vector width: one element per lane, several chunks per lane
    "odd_d1023_260": lambda: (manifolds(n_manifolds=4, per_manifold=65, D=1023, k=3,
                                        noise=0.005, seed=1011)[0],
                              dict(d=7, K_hd=12, K_ld=9, n_neg=5, alpha=1.3, perplexity=6.0)),
    # HD lists longer than a wave (held in LDS): 128 and 256 entries, and 100
    # (not a multiple of 8: the affinity pass scans the whole list) on rows of
    # odd width
    "long_hd128_2000": lambda: (manifolds(n_manifolds=10, per_manifold=200, D=32, k=3,
                                          seed=1012)[0],
                                dict(d=2, K_hd=128, K_ld=16, n_neg=8, alpha=1.0,
                                     perplexity=30.0)),
    "long_hd256_3000_bf16": lambda: (f32_to_bf16_bits(manifolds(n_manifolds=12, per_manifold=250,
                                                                D=64, k=4, seed=1013)[0]),
                                     # 8 times the entries per row of the 32-entry
                                     # cases: 8 times the rows with a tie allowed
                                     dict(d=8, K_hd=256, K_ld=32, n_neg=16, alpha=0.7,
                                          perplexity=50.0, tie_rows=48)),
    "long_hd100_777": lambda: (np.random.default_rng(4).normal(size=(777, 13)).astype(np.float32),
                               dict(d=3, K_hd=100, K_ld=9, n_neg=5, alpha=1.3, perplexity=20.0)),
    # the smallest case: N = 6, one input dimension, d = 1
    "tiny_6": lambda: (np.array([[0.0], [0.3], [1.1], [2.0], [2.2], [5.0]], dtype=np.float32),
                       dict(d=1, K_hd=3, K_ld=2, n_neg=2, alpha=1.0, perplexity=2.0)),
    "odd_dims_777": lambda: (np.random.default_rng(3).normal(size=(777, 13)).astype(np.float32),
                             dict(d=5, K_hd=10, K_ld=7, n_neg=3, alpha=1.7, perplexity=4.0)),
}


def _setup(O, F, name, seed=42, **hpkw):
    X, c = WORKLOADS[name]()
    N = X.shape[0]
    hp_o, hp_g = make_hp(O, F, N, alpha=c["alpha"], perplexity=c["perplexity"],
                         n_neg=c["n_neg"], **hpkw)
    Y0 = y_init(N, c["d"])
    S = O.OracleState(X, c["d"], c["K_hd"], c["K_ld"], seed, Y0).init(hp_o)
    emb = F.Embedding(X, Y0, c["d"], c["K_hd"], c["K_ld"], seed=seed, hp=hp_g)
    return X, c, S, emb, hp_o, hp_g


def _check_hd(X, c, g, S, bf16):
    tol = hd_tie_tol(X.shape[1], bf16)
    N = S.N
    differ, nbad, bad = compare_hd_rows(X, g["hd_idx"], S.live("hd_idx"), S.live("hd_d2"), tol)
    assert nbad == 0, f"HD rows beyond the tie rule: {bad[:10]}"
    assert differ <= (c or {}).get("tie_rows", max(3, N // 500)), f"{differ} HD rows differ at ties"
    same = np.all(g["hd_idx"] == S.live("hd_idx"), axis=1)
    d_o = S.live("hd_d2")[same]
    assert np.all(np.abs(g["hd_d2"][same] - d_o) <= 0.5 * tol * d_o + 1e-30)
    return same


def _clean_points(S, same_hd):
    """Points whose HD row and whose HD neighbours' rows match the oracle exactly.

    A tie-swapped row j changes the neighbour-of-neighbour candidates of every
    point listing j, so those points are compared through properties only.
    """
    hd = S.live("hd_idx")
    return same_hd & np.all(same_hd[hd], axis=1)


def _clean_affinity(S, g_hd, same_hd):
    """Points whose HD row matches and whose neighbours' rows hold the same sets
    (the symmetrised affinity only asks whether i is listed by j)."""
    o_hd = S.live("hd_idx")
    same_set = np.array([set(a.tolist()) == set(b.tolist()) for a, b in zip(g_hd, o_hd)])
    return same_hd & np.all(same_set[o_hd], axis=1)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_init_matches_oracle(oracle_lib, fsne_lib, name):
    O, F = oracle_lib, fsne_lib
    X, c, S, emb, hp_o, hp_g = _setup(O, F, name)
    g = emb.state()
    np.testing.assert_array_equal(g["ld_idx"], S.live("ld_idx"))        # integer draws
    same = _check_hd(X, c, g, S, X.dtype == np.uint16)
    rec_o = np.stack([S.live("beta"), S.live("m"), S.live("r"), S.live("invS")], 1)
    assert rel_l2(g["rec"][same, 0], rec_o[same, 0]) < 1e-4          # beta
    assert rel_l2(g["rec"][same, 3], rec_o[same, 3]) < 1e-4          # invS
    cleanP = _clean_affinity(S, g["hd_idx"], same)
    assert cleanP.mean() > 0.97
    assert rel_l2(g["P"][cleanP], S.live("P")[cleanP]) < 1e-4
    assert g["E"] == 1.0 and g["t"] == 0
    emb.close()


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("hd_mode", [1, 0])
def test_step_matches_oracle_with_injection(oracle_lib, fsne_lib, name, hd_mode):
    """Six iterations, each from the oracle's state injected into the GPU and
    compared phase by phase over every point (tests/parity.py)."""
    O, F = oracle_lib, fsne_lib
    X, c, S, emb, hp_o, hp_g = _setup(O, F, name, hd_mode=hd_mode)
    bf16 = X.dtype == np.uint16
    fired_seen = set()
    n_fired, r0 = 0, emb.stats()["hd_refinements"]
    for it in range(6):
        g, out = check_injected_step(O, S, emb, hp_o, lambda g, S: _check_hd(X, c, g, S, bf16),
                                     tie_rows=c.get("tie_rows"))
        st = emb.stats()
        fired_seen.add(st["last_fired"])
        n_fired += int(st["last_fired"])
        assert st["hd_refinements"] - r0 == n_fired
        # every LD list is a valid list of distinct other points
        ld = g["ld_idx"]
        assert np.all((ld >= 0) & (ld < S.N)) and not np.any(ld == np.arange(S.N)[:, None])
        assert all(len(set(r.tolist())) == ld.shape[1] for r in ld)
        assert g["Y"].shape == (S.N, c["d"])
    if hd_mode == 1:
        assert fired_seen == {1}
    emb.close()


def test_complete_lists_give_the_exact_gradient(oracle_lib, fsne_lib):
    """K_hd = N - 1: the GPU step equals plain gradient descent on eq. (5)."""
    O, F = oracle_lib, fsne_lib
    rng = np.random.default_rng(9)
    N, D, d = 48, 6, 3
    X = rng.normal(size=(N, D)).astype(np.float32)
    Y0 = rng.normal(scale=1.5, size=(N, d)).astype(np.float32)
    for alpha in (0.5, 1.0, 2.5):
        hp_o, hp_g = make_hp(O, F, N, alpha=alpha, perplexity=8.0, lr=2.0, momentum=0.0,
                             attr=1.0, n_neg=4, hd_mode=1)
        emb = F.Embedding(X, Y0, d, N - 1, N - 1, seed=5, hp=hp_g)
        emb.step(1)
        Y1 = emb.Y().astype(np.float64)
        Pex, _ = O.exact_P(X, 8.0)
        G = O.exact_grad(Pex, Y0.astype(np.float64), alpha)
        assert rel_l2(Y1 - Y0, -hp_o.lr * G) < 1e-4
        emb.close()


def test_free_run_recall_and_validity(oracle_lib, fsne_lib):
    """500 GPU iterations on the 2000-point blobs: lists valid, HD recall near 1."""
    O, F = oracle_lib, fsne_lib
    X, lab = blobs(seed=1001)
    N = X.shape[0]
    hp_o, hp_g = make_hp(O, F, N)
    emb = F.Embedding(X, y_init(N, 2), 2, 32, 16, seed=42, hp=hp_g)
    prev_kth = emb.knn(0)[1][:, -1].copy()
    for it in range(25):
        emb.step(20)
        idx, d2 = emb.knn(0)
        assert np.all(np.diff(d2, axis=1) >= 0)
        assert np.all(d2[:, -1] <= prev_kth)
        prev_kth = d2[:, -1].copy()
        if it == 12:
            emb.set_hyperparams(F.fsne_default_hparams(**{**hp_g.as_dict(), "attr": 1.0,
                                                           "momentum": 0.8}))
    idx, d2 = emb.knn(0)
    ld, _ = emb.knn(1)
    for i in range(0, N, 37):
        assert len(set(idx[i])) == 32 and i not in set(idx[i])
        assert len(set(ld[i])) == 16 and i not in set(ld[i])
    ex, _ = O.knn_exact(X, np.arange(N), 32)
    recall = np.mean([len(set(idx[i]) & set(ex[i])) for i in range(N)]) / 32
    assert recall > 0.99, recall
    agree = (lab[ld] == lab[:, None]).mean()
    assert agree > 0.97, agree
    st = emb.stats()
    assert st["status"] == 0 and st["t"] == 500
    emb.close()


def test_determinism_and_resume(fsne_lib, oracle_lib):
    O, F = oracle_lib, fsne_lib
    X, _ = blobs(seed=1001)
    N = X.shape[0]
    _, hp_g = make_hp(O, F, N)
    Y0 = y_init(N, 2)
    a = F.Embedding(X, Y0, 2, 32, 16, seed=7, hp=hp_g)
    b = F.Embedding(X, Y0, 2, 32, 16, seed=7, hp=hp_g)
    a.step(60)
    b.step(60)
    assert np.array_equal(a.Y(), b.Y())
    snap = a.state()
    a.step(40)
    c = F.Embedding(X, Y0, 2, 32, 16, seed=7, hp=hp_g)
    c.set_state({k: v for k, v in snap.items() if k not in ("A", "R", "Zh")})
    c.step(40)
    assert np.array_equal(a.Y(), c.Y())
    assert np.array_equal(a.knn(0)[0], c.knn(0)[0])
    for e in (a, b, c):
        e.close()


def test_perplexity_change_and_implode(oracle_lib, fsne_lib):
    O, F = oracle_lib, fsne_lib
    X, c, S, emb, hp_o, hp_g = _setup(O, F, "blobs_1237")
    emb.step(5)
    st = emb.state()
    hp2 = F.fsne_default_hparams(**{**hp_g.as_dict(), "perplexity": 5.0})
    emb.set_hyperparams(hp2)
    g = emb.state()
    for i in range(0, st["hd_d2"].shape[0], 97):
        (beta, m, r, invS), _ = O.calibrate(g["hd_d2"][i].astype(np.float64), 5.0)
        assert abs(g["rec"][i, 0] - beta) <= 1e-4 * beta
    Y = emb.Y()
    emb.implode(10.0)
    assert np.allclose(emb.Y(), Y / 10.0, rtol=1e-6)
    emb.close()


def test_insert_and_drift_match_oracle(oracle_lib, fsne_lib):
    O, F = oracle_lib, fsne_lib
    X, _ = blobs(seed=1001)
    N0, n_ins = 1500, 300
    hp_o, hp_g = make_hp(O, F, N0, hd_mode=1)
    Y0 = y_init(N0, 2)
    S = O.OracleState(X[:N0], 2, 32, 16, 42, Y0, capacity=N0 + n_ins).init(hp_o)
    emb = F.Embedding(X[:N0], Y0, 2, 32, 16, seed=42, hp=hp_g, capacity=N0 + n_ins)
    for _ in range(3):
        S.step(hp_o)
    emb.set_state(S.as_gpu_state())
    Yn = np.random.default_rng(1).normal(size=(n_ins, 2)).astype(np.float32)
    S.insert(hp_o, X[N0:N0 + n_ins], Yn)
    emb.insert(X[N0:N0 + n_ins], Yn)
    g = emb.state()
    Xall = X[:N0 + n_ins]
    np.testing.assert_array_equal(g["ld_idx"][N0:], S.live("ld_idx")[N0:])
    same = _check_hd(Xall, None, g, S, False)
    clean = _clean_affinity(S, g["hd_idx"], same)
    assert rel_l2(g["P"][clean], S.live("P")[clean]) < 1e-4
    # drift 40 points to new coordinates
    rng = np.random.default_rng(2)
    ids = rng.choice(N0 + n_ins, 40, replace=False)
    Xn = (X[ids] + rng.normal(scale=0.5, size=X[ids].shape)).astype(np.float32)
    Yd = rng.normal(size=(40, 2)).astype(np.float32)
    emb.set_state(S.as_gpu_state())
    S.drift(hp_o, ids, Xn, Yd)
    emb.drift(ids, Xn, Yd)
    g = emb.state()
    Xall = S.X[:S.N]
    same = _check_hd(Xall, None, g, S, False)
    np.testing.assert_array_equal(g["flags"][same], S.live("flags")[same])
    np.testing.assert_allclose(g["Y"][ids], Yd)
    assert np.all(g["V"][ids] == 0)
    clean = _clean_affinity(S, g["hd_idx"], same)
    assert rel_l2(g["P"][clean], S.live("P")[clean]) < 1e-4
    emb.close()


@pytest.mark.parametrize("name", ["manifold_4003_bf16", "zipf_3000_bf16"])
def test_bf16_screen_against_direct_and_oracle(oracle_lib, fsne_lib, name):
    """BF16 form: MFMA expanded-form screen, FP32 direct re-rank of survivors.

    From the same injected state the screened step equals the direct FP32
    step on the same BF16 rows, except in rows where the screen dropped a
    candidate that would have entered the list; those rows are counted and
    must stay rare.  Stored distances are the direct FP32 ones, so they meet
    the oracle's tie rule."""
    O, F = oracle_lib, fsne_lib
    X, c, S, direct, hp_o, hp_g = _setup(O, F, name, hd_mode=1)
    hp_s = F.fsne_default_hparams(**{**hp_g.as_dict(), "dist_mode": 1})
    screened = F.Embedding(X, y_init(X.shape[0], c["d"]), c["d"], c["K_hd"], c["K_ld"], seed=42,
                           hp=hp_s)
    lost_rows = 0
    for it in range(4):
        st0 = S.as_gpu_state()
        direct.set_state(st0)
        screened.set_state(st0)
        S.step(hp_o)
        direct.step(1)
        screened.step(1)
        gd, gs = direct.state(), screened.state()
        differ = ~np.all(gd["hd_idx"] == gs["hd_idx"], axis=1)
        for i in np.where(differ)[0]:
            # the screened row is a valid list that misses candidates the direct row took
            assert len(set(gs["hd_idx"][i].tolist())) == c["K_hd"]
            assert np.all(gs["hd_d2"][i][-1] >= gd["hd_d2"][i][-1])
        lost_rows += int(differ.sum())
        same = ~differ
        np.testing.assert_array_equal(gs["hd_d2"][same], gd["hd_d2"][same])  # same FP32 sums
        tol = hd_tie_tol(X.shape[1], True)
        _, nbad, bad = compare_hd_rows(X, gs["hd_idx"], S.live("hd_idx"), S.live("hd_d2"), tol,
                                       rows=np.where(same)[0])
        assert nbad == 0, bad[:5]
    assert lost_rows <= 0.005 * 4 * X.shape[0], lost_rows
    direct.close()
    screened.close()


@pytest.mark.parametrize("name", ["blobs_2000", "manifold_4003_bf16", "odd_dims_777"])
def test_delete_matches_oracle(oracle_lib, fsne_lib, name):
    """Deleting points: the same renumbering, list rewrite and recalibration
    on both sides, then one more iteration from the reduced state."""
    O, F = oracle_lib, fsne_lib
    X, c, S, emb, hp_o, hp_g = _setup(O, F, name, hd_mode=1)
    for _ in range(3):
        S.step(hp_o)
    emb.set_state(S.as_gpu_state())
    rng = np.random.default_rng(5)
    N0 = S.N
    ids = rng.choice(N0, N0 // 7, replace=False)
    S.delete(hp_o, ids)
    emb.delete(ids)
    assert emb.stats()["N"] == S.N
    g = emb.state()
    Xl = S.X[:S.N]
    np.testing.assert_array_equal(g["Y"], S.live("Y").astype(np.float32))
    np.testing.assert_array_equal(g["ld_idx"], S.live("ld_idx"))
    same = _check_hd(Xl, c, g, S, X.dtype == np.uint16)
    np.testing.assert_array_equal(g["flags"][same], S.live("flags")[same])
    rec_o = np.stack([S.live("beta"), S.live("m"), S.live("r"), S.live("invS")], 1)
    assert rel_l2(g["rec"][same, 0], rec_o[same, 0]) < 1e-4
    clean = _clean_affinity(S, g["hd_idx"], same)
    assert clean.mean() > 0.95
    assert rel_l2(g["P"][clean], S.live("P")[clean]) < 1e-4
    # the next iteration from the reduced state
    emb.set_state(S.as_gpu_state())
    S.step(hp_o)
    emb.step(1)
    g = emb.state()
    same = _check_hd(Xl, c, g, S, X.dtype == np.uint16)
    assert np.all(np.isfinite(g["Y"])) and emb.stats()["nonfinite"] == 0
    emb.close()


def test_long_lists_reach_the_exact_neighbours(oracle_lib, fsne_lib):
    """Lists of 256 on 3,000 blob points: after 400 GPU iterations the HD lists
    hold nearly all exact 256 nearest neighbours and stay valid."""
    O, F = oracle_lib, fsne_lib
    X, lab = blobs(n_clusters=6, per_cluster=500, D=20, seed=1014)
    N, K = X.shape[0], 256
    hp_o, hp_g = make_hp(O, F, N, perplexity=60.0)
    emb = F.Embedding(X, y_init(N, 2), 2, K, 16, seed=42, hp=hp_g)
    emb.step(250)
    emb.set_hyperparams(F.fsne_default_hparams(**{**hp_g.as_dict(), "attr": 1.0,
                                                   "momentum": 0.8}))
    emb.step(150)
    idx, d2 = emb.knn(0)
    assert np.all(np.diff(d2, axis=1) >= 0)
    assert all(len(set(r.tolist())) == K and i not in set(r.tolist()) for i, r in enumerate(idx))
    ex, _ = O.knn_exact(X, np.arange(N), K)
    recall = np.mean([len(set(idx[i]) & set(ex[i])) for i in range(N)]) / K
    assert recall > 0.95, recall
    assert emb.stats()["nonfinite"] == 0
    emb.close()


def test_captured_graph_equals_eager_launches(fsne_lib):
    """fsne_step runs chunks of 25 iterations as one captured HIP graph unless
    kernel timing is on; with timing on every launch goes out on its own.
    Both give the same state bit for bit over several replays, with a
    hyperparameter change (a new capture), a state load and host reads
    between them."""
    F = fsne_lib
    X, _ = blobs(seed=1001)
    N = X.shape[0]
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N / 12.0, attr=12.0, n_neg=8)
    eager = F.Embedding(X, y_init(N, 2), 2, 32, 16, seed=9, hp=hp)
    graph = F.Embedding(X, y_init(N, 2), 2, 32, 16, seed=9, hp=hp)
    eager.profile(True)
    fields = ["Y", "V", "hd_idx", "hd_d2", "ld_idx", "rec", "P", "flags"]
    for k in range(5):
        eager.step(55)      # 2 graph replays + 5 single iterations on the other side
        graph.step(55)
        ge, gg = eager.state(fields), graph.state(fields)
        for f in fields:
            assert np.array_equal(ge[f], gg[f]), (k, f)
        assert eager.stats()["t"] == graph.stats()["t"] == 55 * (k + 1)
        if k == 1:
            hp2 = F.fsne_default_hparams(**{**hp.as_dict(), "attr": 1.0, "momentum": 0.8})
            eager.set_hyperparams(hp2)
            graph.set_hyperparams(hp2)
        if k == 2:
            s = graph.state()
            graph.set_state({f: v for f, v in s.items() if f not in ("A", "R", "Zh")})
            s = eager.state()
            eager.set_state({f: v for f, v in s.items() if f not in ("A", "R", "Zh")})
    eager.close()
    graph.close()
