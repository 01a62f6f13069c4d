"""Jump start by a random linear projection (Sec. 3): the GPU projection
equals the oracle's, and starting the lists from a projected embedding
improves the HD lists faster than from a random one."""
import numpy as np
import pytest

from inputs.generators import blobs, f32_to_bf16_bits, make_workload, y_init
from inputs.knn_metrics import exact_knn, rnx_auc, rnx_curve
from tests.parity import rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

CASES = {
    "blobs_f32_d2": lambda: (blobs(seed=1001)[0], 2),
    "manifold_bf16_d16": lambda: (f32_to_bf16_bits(make_workload("manifold_1m", N=4003)[0]), 16),
    "odd_f32_d5": lambda: (np.random.default_rng(3).normal(size=(777, 13)).astype(np.float32), 5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_jump_start_matches_oracle(oracle_lib, fsne_lib, case):
    O, F = oracle_lib, fsne_lib
    X, d = CASES[case]()
    N = X.shape[0]
    emb = F.Embedding(X, y_init(N, d), d, 10, 7, seed=42,
                      hp=F.fsne_default_hparams(perplexity=4.0, n_neg=4))
    S = O.OracleState(X, d, 10, 7, 42, y_init(N, d))
    for projection, sigma in ((0, 1e-2), (3, 2.5)):
        emb.jump_start(projection, sigma)
        S.jump_start(projection, sigma)
        g = emb.state(["Y", "V"])
        assert np.all(g["V"] == 0.0)
        assert rel_l2(g["Y"], S.live("Y")) < 1e-5, (case, projection)
    emb.close()


def test_jump_start_speeds_up_the_hd_lists(fsne_lib):
    F = fsne_lib
    X, _, _ = make_workload("manifold_1m", N=6000)
    N, d, K = X.shape[0], 2, 32
    q = np.arange(0, N, 7)
    ex, _ = exact_knn(X, q, K)
    auc = {}
    for mode in ("random", "projected"):
        hp = F.fsne_default_hparams(perplexity=10.0, lr=0.0, n_neg=16)
        emb = F.Embedding(X, y_init(N, d), d, K, K, seed=3, hp=hp)
        if mode == "projected":
            emb.jump_start(0, 1e-2)
        emb.step(40)          # learning rate 0: the embedding stays as it is
        idx, _ = emb.knn(0)
        auc[mode] = rnx_auc(rnx_curve(idx[q], ex, N))
        emb.close()
    print("AUC of R_NX after 40 iterations, fixed embedding", auc)
    assert auc["projected"] > auc["random"] + 0.01, auc
