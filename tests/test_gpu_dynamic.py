"""Dynamic data with learned placement (scaled version of the 500k-point
insertion workload): new points placed by the trained network reach the
LD neighbour recall target in fewer iterations than points placed at random.

The rows come from the styled image-like generator (a 3-dimensional style
manifold within each class), as in the benchmark's online-use leg: with
independent pixel drops the exact neighbours have no low-dimensional
structure, the base embedding's recall sits near chance, and a target
derived from it does not separate the two placements."""
import numpy as np
import pytest

from inputs.generators import image_styles, y_init
from inputs.knn_metrics import exact_knn

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def ld_recall(Y, rows, hd_nn, K):
    """Mean fraction of each row's exact LD K-NN (in Y) that are among its exact HD K-NN."""
    Yd = Y.astype(np.float64)
    hits = 0
    for a, i in enumerate(rows):
        dd = ((Yd - Yd[i]) ** 2).sum(1)
        dd[i] = np.inf
        nn = np.argpartition(dd, K)[:K]
        hits += len(set(nn.tolist()) & set(hd_nn[a].tolist()))
    return hits / (len(rows) * K)


def test_learned_placement_beats_random_init(fsne_lib):
    F = fsne_lib
    N0, n_new, K = 12000, 1200, 32
    classes = np.random.default_rng(1004).integers(0, 10, N0 + n_new)
    X, _ = image_styles(classes, seed=1004, proto_seed=1002)
    Xb, Xn = X[:N0], X[N0:N0 + n_new]
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N0 / 12.0, attr=12.0, n_neg=16)
    base = F.Embedding(Xb, y_init(N0, 2), 2, K, K, seed=5, hp=hp)
    base.step(250)
    hp2 = F.fsne_default_hparams(**{**hp.as_dict(), "attr": 1.0, "momentum": 0.8})
    base.set_hyperparams(hp2)
    base.step(350)
    snap = {k: v for k, v in base.state().items() if k not in ("A", "R", "Zh")}
    net = F.Mlp(base, F.fsne_mlp_default_opts(epochs=40, batch=1024))
    net.train(base)
    rows_b = np.arange(0, N0, N0 // 300)
    hd_b, _ = exact_knn(X[:N0], rows_b, K)
    target = 0.9 * ld_recall(base.Y(), rows_b, hd_b, K)
    rows = np.arange(N0, N0 + n_new, 4)
    hd_nn, _ = exact_knn(X[:N0 + n_new], rows, K)
    iters = {}
    for mode in ("mlp", "random"):
        emb = F.Embedding(Xb, y_init(N0, 2), 2, K, K, seed=5, hp=hp2, capacity=N0 + n_new)
        emb.set_state(snap)
        Yn = net.predict(Xn) if mode == "mlp" else y_init(n_new, 2, seed=99)
        emb.insert(Xn, Yn)
        reached = None
        for it in range(0, 601, 10):
            if ld_recall(emb.Y(), rows, hd_nn, K) >= target:
                reached = it
                break
            emb.step(10)
        iters[mode] = 10_000 if reached is None else reached
        emb.close()
    print("iterations to the recall target", iters, "target", target)
    assert iters["mlp"] <= 600 and iters["mlp"] < iters["random"], iters
    net.close()
    base.close()
