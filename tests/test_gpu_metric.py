"""The angular HD metric and a live metric switch against the oracle.

Under the angular metric the GPU computes each row's scale 1/|x| in FP32, so
every unit row carries a common relative error eta <= eps = (D/2 + 3) u
(u = 2^-24: the norm's D-term sum, the square root, the reciprocal and the
product).  To first order the squared distance of two unit rows then moves by
2 (x - y).(eta_x x - eta_y y) <= 4 eps sqrt(d2), on top of the summation
error gamma d2 of the Euclidean kernels.  Two list entries may swap when
their exact distances are closer than twice that, and the affinities, which
go as exp(-beta d2), may differ by beta times it: a few 1e-4 relative at the
closest pairs, hence the 1e-3 bound on P, the gradient partials and the step
(1e-4 for the Euclidean metric).
"""
import numpy as np
import pytest

from inputs.generators import f32_to_bf16_bits, bf16_bits_to_f32, image_like, manifolds, y_init, \
    zipf_mixture
from tests.parity import check_injected_step, hd_tie_tol, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

U = 2.0 ** -24


def _rescale(X, seed):
    """Rows scaled by powers of two (exact): angular and Euclidean neighbours differ."""
    rng = np.random.default_rng(seed)
    return (X * np.exp2(rng.integers(-3, 4, size=(X.shape[0], 1)))).astype(np.float32)


# name: (rows, d, K_hd, K_ld, n_neg)
CASES = {
    # two points per wave (FP32 unit rows of 128)
    "manifold_2000_f32": (lambda: _rescale(manifolds(per_manifold=40, seed=1003)[0], 7),
                          2, 32, 16, 8),
    # one point per wave (K_hd = 64), BF16 rows widened to FP32 unit rows of 256
    "zipf_1500_bf16_k64": (lambda: f32_to_bf16_bits(_rescale(
        zipf_mixture(N=1500, n_clusters=20, seed=1005)[0], 9)), 4, 64, 32, 16),
    # one point per wave over four row chunks (784 wide)
    "image_1200_f32": (lambda: _rescale(image_like(n_per_class=120, seed=1011)[0], 11),
                       2, 32, 16, 8),
}


def _unit(X):
    Xf = (bf16_bits_to_f32(X) if X.dtype == np.uint16 else X).astype(np.float64)
    n = np.sqrt((Xf * Xf).sum(1, keepdims=True))
    return np.where(n > 0, Xf / np.where(n > 0, n, 1.0), 0.0)


def _tol(D, d2):
    """Bound on |GPU d2 - exact d2| (see the module docstring)."""
    eps = (D / 2 + 3) * U
    return 4.0 * eps * np.sqrt(np.maximum(d2, 0.0)) + 0.5 * hd_tie_tol(D) * d2


def _check_lists(Xu, D, g_idx, g_d2, o_idx, o_d2, max_differ):
    """Rows equal, or differing only where exact angular distances tie within
    twice the bound; equal rows carry distances within the bound."""
    N = g_idx.shape[0]
    differ = 0
    for i in range(N):
        gi, oi = g_idx[i], o_idx[i]
        if np.array_equal(gi, oi):
            assert np.all(np.abs(g_d2[i] - o_d2[i]) <= _tol(D, o_d2[i]) + 1e-30), i
            continue
        differ += 1
        assert len(set(gi.tolist())) == len(gi) and i not in set(gi.tolist()), i
        ex = ((Xu[gi] - Xu[i]) ** 2).sum(1)
        assert np.all(np.abs(ex - o_d2[i]) <= 2.0 * _tol(D, o_d2[i]) + 1e-30), i
    assert differ <= max_differ, differ
    return np.all(g_idx == o_idx, axis=1)


def _setup(O, F, name, metric, hd_mode=1, seed=42):
    X = CASES[name][0]()
    d, Kh, Kl, nneg = CASES[name][1:]
    N = X.shape[0]
    base = dict(alpha=1.0, perplexity=10.0, lr=N / 12.0, momentum=0.5, attr=12.0, rep=1.0,
                n_neg=nneg, hd_mode=hd_mode, e_smooth=0.1, p_min=0.05)
    hp_o = O.Hyper(**{k: (float(np.float32(v)) if isinstance(v, float) else v)
                      for k, v in base.items()})
    hp_g = F.fsne_default_hparams(**base, metric=metric)
    Y0 = y_init(N, d)
    S = O.OracleState(X, d, Kh, Kl, seed, Y0, metric=metric).init(hp_o)
    emb = F.Embedding(X, Y0, d, Kh, Kl, seed=seed, hp=hp_g)
    return X, S, emb, hp_o, hp_g


def _clean(S, same):
    hd = S.live("hd_idx")
    return same & np.all(same[hd], axis=1)


@pytest.mark.parametrize("name", list(CASES))
def test_angular_init_and_steps_match_oracle(oracle_lib, fsne_lib, name):
    O, F = oracle_lib, fsne_lib
    X, S, emb, hp_o, hp_g = _setup(O, F, name, metric=1)
    D, N = X.shape[1], X.shape[0]
    Xu = _unit(X)
    assert emb.hyperparams().metric == 1
    g = emb.state()
    same = _check_lists(Xu, D, g["hd_idx"], g["hd_d2"], S.live("hd_idx"), S.live("hd_d2"),
                        max(3, N // 200))
    # the initial lists are the same random draws, sorted by the angular distance
    assert all(set(a.tolist()) == set(b.tolist()) for a, b in zip(g["hd_idx"], S.live("hd_idx")))
    assert rel_l2(g["rec"][same, 0], S.live("beta")[same]) < 1e-3
    for _ in range(4):
        g, out = check_injected_step(
            O, S, emb, hp_o, fp_tol=1e-3, tie_rows=max(3, N // 200),
            check_hd=lambda g, S: _check_lists(Xu, D, g["hd_idx"], g["hd_d2"], S.live("hd_idx"),
                                               S.live("hd_d2"), max(3, N // 200)))
        assert out["fired"] == 1
    emb.close()


@pytest.mark.parametrize("name", list(CASES))
def test_metric_switch_matches_oracle(oracle_lib, fsne_lib, name):
    """Euclidean for a few steps, then the angular metric on both sides: the
    same members per list, distances in the new metric, sorted, calibrated,
    flagged, E = 1, matching affinities; a step after it; then back."""
    O, F = oracle_lib, fsne_lib
    X, S, emb, hp_o, hp_g = _setup(O, F, name, metric=0, hd_mode=0)
    D, N = X.shape[1], X.shape[0]
    Xu = _unit(X)
    for _ in range(3):
        S.step(hp_o)
    emb.set_state(S.round_to_f32().as_gpu_state())
    before = S.live("hd_idx").copy()
    S.set_metric(hp_o, 1)
    emb.set_hyperparams(F.fsne_default_hparams(**{**hp_g.as_dict(), "metric": 1}))
    g = emb.state()
    assert g["E"] == 1.0 and S.E[0] == 1.0
    assert np.all(g["flags"] & 1) and np.all(S.live("flags") == 1)
    for i in range(N):
        assert set(g["hd_idx"][i].tolist()) == set(before[i].tolist())
        assert np.all(np.diff(g["hd_d2"][i]) >= 0)
    same = _check_lists(Xu, D, g["hd_idx"], g["hd_d2"], S.live("hd_idx"), S.live("hd_d2"),
                        max(3, N // 200))
    assert rel_l2(g["rec"][same, 0], S.live("beta")[same]) < 1e-3
    clean = same & np.all(same[S.live("hd_idx")], axis=1)
    assert clean.mean() > 0.9
    assert rel_l2(g["P"][clean], S.live("P")[clean]) < 1e-3
    assert emb.stats()["next_fire"] == 1        # E = 1: the next step refines
    # one step under the new metric, from the same state
    emb.set_state(S.as_gpu_state())
    out = S.step(hp_o)
    emb.step(1)
    g = emb.state()
    assert out["fired"] == 1 and emb.stats()["last_fired"] == 1
    _check_lists(Xu, D, g["hd_idx"], g["hd_d2"], S.live("hd_idx"), S.live("hd_d2"),
                 max(3, N // 200))
    # back to the Euclidean metric
    emb.set_state(S.as_gpu_state())
    S.set_metric(hp_o, 0)
    emb.set_hyperparams(F.fsne_default_hparams(**{**hp_g.as_dict(), "metric": 0}))
    g = emb.state()
    Xf = (bf16_bits_to_f32(X) if X.dtype == np.uint16 else X).astype(np.float64)
    for i in range(0, N, 7):
        ex = ((Xf[g["hd_idx"][i]] - Xf[i]) ** 2).sum(1)
        assert np.all(np.abs(g["hd_d2"][i] - ex) <= hd_tie_tol(D, X.dtype == np.uint16) * ex)
    emb.close()


def test_angular_rejects_the_screen(fsne_lib):
    F = fsne_lib
    X = f32_to_bf16_bits(np.random.default_rng(0).normal(size=(300, 32)).astype(np.float32))
    hp = F.fsne_default_hparams(dist_mode=1, metric=1, perplexity=5.0)
    with pytest.raises(F.FsneError) as e:
        F.Embedding(X, y_init(300, 2), 2, 16, 8, seed=1, hp=hp)
    assert e.value.status == F.FSNE_EINVAL
    emb = F.Embedding(X, y_init(300, 2), 2, 16, 8, seed=1,
                      hp=F.fsne_default_hparams(dist_mode=1, perplexity=5.0))
    with pytest.raises(F.FsneError):
        emb.set_hyperparams(F.fsne_default_hparams(dist_mode=1, metric=1, perplexity=5.0))
    assert emb.hyperparams().metric == 0
    emb.close()


def test_angular_insert_drift_delete_match_oracle(oracle_lib, fsne_lib):
    """Online use under the angular metric: inserted rows get lists sorted by
    the angular distance, drifted rows have their unit rows and every
    distance involving them recomputed, deleted rows' refills get angular
    distances; each time the GPU state matches the oracle's."""
    O, F = oracle_lib, fsne_lib
    X_all = _rescale(manifolds(per_manifold=44, seed=1003)[0], 7)      # 2,200 rows
    N0, n_ins = 2000, 200
    base = dict(alpha=1.0, perplexity=10.0, lr=N0 / 12.0, momentum=0.5, attr=12.0, rep=1.0,
                n_neg=8, hd_mode=1, e_smooth=0.1, p_min=0.05)
    hp_o = O.Hyper(**{k: (float(np.float32(v)) if isinstance(v, float) else v)
                      for k, v in base.items()})
    hp_g = F.fsne_default_hparams(**base, metric=1)
    Y0 = y_init(N0, 2)
    S = O.OracleState(X_all[:N0], 2, 32, 16, 42, Y0, capacity=N0 + n_ins, metric=1).init(hp_o)
    emb = F.Embedding(X_all[:N0], Y0, 2, 32, 16, seed=42, hp=hp_g, capacity=N0 + n_ins)
    for _ in range(3):
        S.step(hp_o)
    D = X_all.shape[1]

    def check():
        g = emb.state()
        Xu = _unit(S.X[:S.N])
        same = _check_lists(Xu, D, g["hd_idx"], g["hd_d2"], S.live("hd_idx"), S.live("hd_d2"),
                            max(3, S.N // 200))
        clean = _clean(S, same)
        assert clean.mean() > 0.8
        assert rel_l2(g["P"][clean], S.live("P")[clean]) < 1e-3
        return g, same

    emb.set_state(S.as_gpu_state())
    Yn = np.random.default_rng(1).normal(size=(n_ins, 2)).astype(np.float32)
    S.insert(hp_o, X_all[N0:], Yn)
    emb.insert(X_all[N0:], Yn)
    g, _ = check()
    np.testing.assert_array_equal(g["ld_idx"][N0:], S.live("ld_idx")[N0:])
    rng = np.random.default_rng(2)
    ids = rng.choice(N0 + n_ins, 40, replace=False)
    Xn = _rescale((X_all[ids] + rng.normal(scale=0.3, size=X_all[ids].shape)).astype(np.float32), 3)
    emb.set_state(S.as_gpu_state())
    S.drift(hp_o, ids, Xn)
    emb.drift(ids, Xn)
    g, same = check()
    np.testing.assert_array_equal(g["flags"][same] & 1, S.live("flags")[same])
    dead = rng.choice(N0 + n_ins, 60, replace=False)
    emb.set_state(S.as_gpu_state())
    S.delete(hp_o, dead)
    emb.delete(dead)
    assert emb.stats()["N"] == S.N
    check()
    emb.close()
