"""Full-size checks of the online and hierarchy entry points at 10^6 points
(the benchmark's workload size): jump start, deletion and clustering give
the oracle's results on the same seeded inputs; the memory of rejected HD
candidates changes no result at this size."""
import numpy as np
import pytest

from inputs.generators import make_workload, y_init
from tests.parity import compare_hd_rows, hd_tie_tol, rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def manifold():
    X, _, cfg = make_workload("manifold_1m")
    return X, cfg


def _hp(O, F, N, cfg):
    kw = dict(alpha=1.0, perplexity=10.0, lr=float(np.float32(N / 12.0)), momentum=0.5,
              attr=12.0, rep=1.0, n_neg=cfg["n_neg"], hd_mode=1, e_smooth=0.1, p_min=0.05)
    return O.Hyper(**kw), F.fsne_default_hparams(**kw)


def test_fullsize_jump_start(oracle_lib, fsne_lib, manifold):
    O, F = oracle_lib, fsne_lib
    X, cfg = manifold
    N, d = X.shape[0], cfg["d"]
    emb = F.Embedding(X, y_init(N, d), d, cfg["K_hd"], cfg["K_ld"], seed=42,
                      hp=F.fsne_default_hparams(n_neg=cfg["n_neg"]))
    S = O.OracleState(X, d, cfg["K_hd"], cfg["K_ld"], 42, y_init(N, d))
    emb.jump_start(1, 1e-2)
    S.jump_start(1, 1e-2)
    g = emb.state(["Y", "V"])
    assert rel_l2(g["Y"], S.live("Y")) < 1e-5
    assert np.all(g["V"] == 0.0)
    emb.close()


def test_fullsize_memo_changes_no_result(fsne_lib, manifold):
    """At the benchmark's size and launch configuration (10^6 FP32 rows, two
    points per wave, 64 remembered rejections): 30 refining iterations with
    the memory of rejected candidates on and off give the same state bit for
    bit, and the memory reads fewer candidate rows."""
    F = fsne_lib
    X, cfg = manifold
    N, d = X.shape[0], cfg["d"]
    fields = ["hd_idx", "hd_d2", "ld_idx", "Y", "P", "rec"]
    out = {}
    for memo in (1, 0):
        hp = F.fsne_default_hparams(alpha=1.0, perplexity=10.0, lr=N / 12.0, momentum=0.5,
                                    attr=12.0, n_neg=cfg["n_neg"], hd_mode=1, reject_memo=memo)
        emb = F.Embedding(X, y_init(N, d), d, cfg["K_hd"], cfg["K_ld"], seed=42, hp=hp)
        emb.step(30)
        st = emb.stats()
        assert st["nonfinite"] == 0
        g = emb.state(fields)
        out[memo] = ({k: g[k].copy() for k in fields}, st["hd_cand_rows"], st["E"])
        emb.close()
    for k in fields:
        assert np.array_equal(out[1][0][k], out[0][0][k]), k
    assert out[1][2] == out[0][2]
    assert out[1][1] < out[0][1], (out[1][1], out[0][1])


def test_fullsize_delete(oracle_lib, fsne_lib, manifold):
    O, F = oracle_lib, fsne_lib
    X, cfg = manifold
    N, d = X.shape[0], cfg["d"]
    hp_o, hp_g = _hp(O, F, N, cfg)
    S = O.OracleState(X, d, cfg["K_hd"], cfg["K_ld"], 42, y_init(N, d)).init(hp_o)
    emb = F.Embedding(X, y_init(N, d), d, cfg["K_hd"], cfg["K_ld"], seed=42, hp=hp_g)
    emb.set_state(S.as_gpu_state())
    ids = np.random.default_rng(6).choice(N, 10_000, replace=False)
    S.delete(hp_o, ids)
    emb.delete(ids)
    g = emb.state(["Y", "hd_idx", "hd_d2", "ld_idx", "rec"])
    np.testing.assert_array_equal(g["ld_idx"], S.live("ld_idx"))
    np.testing.assert_array_equal(g["Y"], S.live("Y").astype(np.float32))
    tol = hd_tie_tol(X.shape[1])
    rows = np.random.default_rng(7).choice(S.N, 20_000, replace=False)
    differ, nbad, bad = compare_hd_rows(S.X[:S.N], g["hd_idx"], S.live("hd_idx"),
                                        S.live("hd_d2"), tol, rows=rows)
    assert nbad == 0, bad[:10]
    same = np.all(g["hd_idx"][rows] == S.live("hd_idx")[rows], axis=1)
    assert rel_l2(g["rec"][rows][same, 0], S.live("beta")[rows][same]) < 1e-4
    emb.close()


def test_fullsize_cluster(oracle_lib, fsne_lib):
    """10^6 points in 16-D around 500 centres, each LD list drawn from the
    point's own group (seeded lists, not the method's): labels equal."""
    O, F = oracle_lib, fsne_lib
    rng = np.random.default_rng(8)
    N, d, K, G = 1_000_000, 16, 32, 500
    group = rng.integers(0, G, N)
    cent = rng.normal(scale=20.0, size=(G, d))
    Y = (cent[group] + rng.normal(scale=0.5, size=(N, d))).astype(np.float32)
    order = np.argsort(group, kind="stable")
    start = np.searchsorted(group[order], np.arange(G))
    size = np.bincount(group, minlength=G)
    lists = np.empty((N, K), np.int32)
    for i in range(0, N, 100_000):
        sl = slice(i, min(N, i + 100_000))
        gi = group[sl]
        pick = start[gi][:, None] + (rng.random((gi.size, K)) * size[gi][:, None]).astype(np.int64)
        lists[sl] = order[pick]
    own = lists == np.arange(N)[:, None]
    lists[own] = (lists[own] + 1) % N            # no self entries (a stray link is fine)
    eps = 3.5        # same-group pairs lie about 2.8 apart in 16-D
    X = np.zeros((N, 4), np.float32)
    emb = F.Embedding(X + rng.normal(size=X.shape).astype(np.float32), y_init(N, d), d, 8, K,
                      seed=3, hp=F.fsne_default_hparams(perplexity=4.0, n_neg=4))
    emb.set_state({"Y": Y, "ld_idx": lists})
    lab_g, nc_g = emb.cluster(eps, 10)
    S = O.OracleState(X, d, 8, K, 3, Y)
    S.ld_idx[:N] = lists
    lab_o, nc_o = S.cluster(eps, 10)
    assert nc_g == nc_o and nc_g > 100
    np.testing.assert_array_equal(lab_g, lab_o)
    emb.close()
