"""Clustering for the hierarchy graph (Sec. 4.2): DBSCAN on the LD
neighbour lists.  The same seeded embedding and lists go to the GPU and to
the oracle; the labels (integer work) must agree exactly."""
import numpy as np
import pytest

from inputs.generators import y_init

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def _embedding(seed, N_per=500, d=4, noise=200):
    rng = np.random.default_rng(seed)
    cent = rng.normal(scale=8.0, size=(6, d))
    Y = np.concatenate([c + rng.normal(scale=s, size=(N_per, d))
                        for c, s in zip(cent, (0.3, 0.5, 0.7, 0.4, 0.6, 0.3))] +
                       [rng.uniform(-20, 20, size=(noise, d))]).astype(np.float32)
    return Y[rng.permutation(Y.shape[0])]


@pytest.mark.parametrize("exact_lists", [True, False])
@pytest.mark.parametrize("min_pts", [3, 8])
def test_cluster_matches_oracle(oracle_lib, fsne_lib, exact_lists, min_pts):
    O, F = oracle_lib, fsne_lib
    Y = _embedding(4)
    N, d, K = Y.shape[0], Y.shape[1], 16
    D2 = ((Y[:, None, :].astype(np.float64) - Y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D2, np.inf)
    lists = np.argsort(D2, axis=1, kind="stable")[:, :K].astype(np.int32)
    rng = np.random.default_rng(9)
    if not exact_lists:      # approximate lists: a fifth of the entries replaced
        for i in range(N):
            for k in rng.choice(K, K // 5, replace=False):
                c = int(rng.integers(N))
                while c == i or c in lists[i]:
                    c = int(rng.integers(N))
                lists[i, k] = c
    kth = np.sqrt(np.sort(D2, axis=1)[:, 4])
    eps = float(np.float32(1.3 * np.median(kth)))
    X = np.zeros((N, 8), np.float32)
    emb = F.Embedding(X + rng.normal(size=X.shape).astype(np.float32), y_init(N, d), d, 8, K,
                      seed=3, hp=F.fsne_default_hparams(perplexity=4.0, n_neg=4))
    emb.set_state({"Y": Y, "ld_idx": lists})
    lab_g, nc_g = emb.cluster(eps, min_pts)
    S = O.OracleState(X, d, 8, K, 3, Y)
    S.ld_idx[:N] = lists
    lab_o, nc_o = S.cluster(eps, min_pts)
    assert nc_g == nc_o and nc_g >= 6
    np.testing.assert_array_equal(lab_g, lab_o)
    emb.close()
