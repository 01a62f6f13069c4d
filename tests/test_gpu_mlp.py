"""Placement network on the GPU vs the FP64 oracle with BF16-rounded operands.

The oracle rounds exactly the operands the matrix cores see; the two sides
differ by accumulation order and by rare round-to-bf16 decisions of
intermediate activations that sit on a rounding boundary.  Measured on the
784 -> 512 -> 512 -> 2 network over 2,048 rows: 1.9e-5 relative L2 on the
first layer's weights (the largest), 1.0e-5 over all parameters; the bound
is 1e-4 per block.
"""
import numpy as np
import pytest

from inputs.generators import blobs, image_like, y_init
from tests.parity import rel_l2

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


def _ctx(F, X, d, K=8):
    return F.Embedding(X, y_init(X.shape[0], d), d, K, min(K, 4), seed=3,
                       hp=F.fsne_default_hparams(perplexity=4.0, n_neg=4))


def _blocks(m_or, flat):
    return m_or.split(np.asarray(flat, dtype=np.float64))


@pytest.mark.parametrize("shape", [(50, 96, 80, 2, 300), (784, 512, 512, 2, 2048),
                                   (128, 64, 48, 16, 517)])
def test_mlp_gradient_matches_oracle(oracle_lib, fsne_lib, shape):
    O, F = oracle_lib, fsne_lib
    D, H1, H2, d, n = shape
    if D == 784:
        X = image_like(n_per_class=-(-n // 10), seed=1002)[0][:n]
    else:
        X = np.random.default_rng(D).normal(size=(n, D)).astype(np.float32)
    T = np.random.default_rng(1).normal(size=(n, d)).astype(np.float32)
    emb = _ctx(F, X, d)
    net = F.Mlp(emb, F.fsne_mlp_default_opts(hidden1=H1, hidden2=H2, batch=max(n, 64), seed=9))
    ora = O.Mlp(D, H1, H2, d, seed=9)
    p, _, _ = net.params()
    np.testing.assert_array_equal(p, ora.params)          # He-uniform init, bit for bit
    # move off the initial point so that biases are non-zero
    p2 = p + np.random.default_rng(2).normal(scale=0.02, size=p.size).astype(np.float32)
    net.set_params(p2)
    ora.params = p2.copy()
    loss_g, g_g = net.loss_grad(X, T)
    loss_o, g_o = ora.loss_grad(X, T, bf16_ops=True)
    assert abs(loss_g - loss_o) <= 1e-4 * loss_o
    errs = {name: rel_l2(bg, bo) for name, bg, bo in
            zip(("W1", "b1", "W2", "b2", "W3", "b3"), _blocks(ora, g_g), _blocks(ora, g_o))}
    print(f"mlp {shape}: loss rel {abs(loss_g - loss_o) / loss_o:.2e}, "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f", all {rel_l2(g_g, g_o):.2e}", flush=True)
    for name, e in errs.items():
        assert e < 1e-4, (name, e)
    assert rel_l2(g_g, g_o) < 1e-4
    net.close()
    emb.close()


def test_mlp_adam_step_and_prediction(oracle_lib, fsne_lib):
    O, F = oracle_lib, fsne_lib
    D, H1, H2, d, n = 50, 64, 64, 2, 256
    X = np.random.default_rng(5).normal(size=(n, D)).astype(np.float32)
    T = np.random.default_rng(6).normal(size=(n, d)).astype(np.float32)
    emb = _ctx(F, X, d)
    net = F.Mlp(emb, F.fsne_mlp_default_opts(hidden1=H1, hidden2=H2, batch=n, seed=4))
    ora = O.Mlp(D, H1, H2, d, seed=4)
    p0 = ora.params.copy()
    net.train_batch(X, T)
    _, g = ora.loss_grad(X, T, bf16_ops=True)
    ora.adam(g)
    p1, _, _ = net.params()
    step_g = p1.astype(np.float64) - p0
    step_o = ora.params.astype(np.float64) - p0
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert big.sum() > 100
    np.testing.assert_allclose(step_g[big], step_o[big], rtol=1e-3, atol=1e-8)
    # prediction: de-standardised forward pass
    mu = np.array([0.5, -2.0], np.float32)
    sd = np.array([3.0, 0.25], np.float32)
    net.set_params(ora.params, mu, sd)
    Yg = net.predict(X)
    Yo = ora.forward(X, bf16_ops=True) * sd + mu
    assert rel_l2(Yg, Yo) < 1e-4
    net.close()
    emb.close()


def test_mlp_fit_to_an_embedding(fsne_lib):
    """Trained on a converged embedding, the network places unseen points
    near their own cluster (the embedding it was fitted to)."""
    F = fsne_lib
    X, lab = blobs(n_clusters=10, per_cluster=400, D=50, seed=21)
    N = 3600
    Xb, lb = X[:N], lab[:N]
    hp = F.fsne_default_hparams(perplexity=10.0, lr=N / 12.0, attr=12.0, n_neg=8)
    emb = F.Embedding(Xb, y_init(N, 2), 2, 32, 16, seed=1, hp=hp)
    emb.step(250)
    emb.set_hyperparams(F.fsne_default_hparams(**{**hp.as_dict(), "attr": 1.0, "momentum": 0.8}))
    emb.step(250)
    Y = emb.Y()
    net = F.Mlp(emb, F.fsne_mlp_default_opts(epochs=60, batch=512, lr=2e-3))
    loss = net.train(emb)
    assert loss < 0.1, loss          # on standardised targets: 90 % of the variance explained
    Yn = net.predict(X[N:])
    cent = np.stack([Y[lb == c].mean(0) for c in range(10)])
    nearest = lambda Z: np.argmin(((Z[:, None, :] - cent[None]) ** 2).sum(-1), axis=1)
    acc_base = (nearest(Y) == lb).mean()          # the embedding's own points
    acc_new = (nearest(Yn) == lab[N:]).mean()     # unseen points placed by the network
    assert acc_base > 0.95 and acc_new > 0.9, (acc_new, acc_base)   # chance is 0.1
    net.close()
    emb.close()
