"""Pins of the placement-MLP oracle (finite differences, rounding, Adam)."""
import numpy as np
import pytest

from inputs.generators import bf16_bits_to_f32, f32_to_bf16_bits


def _small(O, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(40, 12)).astype(np.float32)
    T = rng.normal(size=(40, 2)).astype(np.float32)
    m = O.Mlp(12, 16, 8, 2, seed=seed)
    m.params += rng.normal(scale=0.05, size=m.np).astype(np.float32)   # non-zero biases
    return X, T, m


def test_mlp_gradient_matches_finite_differences(oracle_lib):
    O = oracle_lib
    X, T, m = _small(O)
    loss, g = m.loss_grad(X, T, bf16_ops=False)
    rng = np.random.default_rng(1)
    h = 1e-3
    base = m.params.copy()
    for k in rng.choice(m.np, 40, replace=False):
        m.params = base.copy()
        m.params[k] = np.float32(base[k] + h)
        hp = float(np.float64(m.params[k]) - np.float64(base[k]))
        lp, _ = m.loss_grad(X, T, bf16_ops=False)
        m.params[k] = np.float32(base[k] - h)
        hm = float(np.float64(base[k]) - np.float64(m.params[k]))
        lm, _ = m.loss_grad(X, T, bf16_ops=False)
        fd = (lp - lm) / (hp + hm)
        assert abs(fd - g[k]) <= 2e-5 * max(1.0, abs(g[k])) + 1e-7, (k, fd, g[k])
    m.params = base


def test_mlp_forward_is_the_stated_network(oracle_lib):
    """Two ReLU layers then a linear one, checked with numpy matmuls."""
    O = oracle_lib
    X, T, m = _small(O)
    W1, b1, W2, b2, W3, b3 = [a.astype(np.float64) for a in m.split()]
    h1 = np.maximum(X.astype(np.float64) @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    out = h2 @ W3.T + b3
    np.testing.assert_allclose(m.forward(X, bf16_ops=False), out, rtol=1e-12, atol=1e-12)
    loss, _ = m.loss_grad(X, T, bf16_ops=False)
    assert abs(loss - np.mean((out - T) ** 2)) < 1e-12


def test_bf16_operand_rounding(oracle_lib):
    """With bf16_ops the big products see round-to-nearest-even bfloat16 operands."""
    O = oracle_lib
    X, T, m = _small(O)
    Xb = bf16_bits_to_f32(f32_to_bf16_bits(X)).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = [a.astype(np.float64) for a in m.split()]
    rb = lambda a: bf16_bits_to_f32(f32_to_bf16_bits(np.asarray(a, np.float32))).astype(np.float64)
    h1 = np.maximum(Xb @ rb(W1).T + b1, 0)
    h2 = np.maximum(rb(h1) @ rb(W2).T + b2, 0)
    out = h2 @ W3.T + b3
    np.testing.assert_allclose(m.forward(X, bf16_ops=True), out, rtol=1e-12, atol=1e-12)


def test_he_uniform_init(oracle_lib):
    O = oracle_lib
    m = O.Mlp(784, 512, 512, 2, seed=11)
    W1, b1, W2, b2, W3, b3 = m.split()
    for W, fan in ((W1, 784), (W2, 512), (W3, 512)):
        bound = np.sqrt(6.0 / fan)
        assert np.all(np.abs(W) <= bound)
        assert abs(W.mean()) < 0.02 * bound
        assert abs(W.var() - bound ** 2 / 3) < 0.02 * bound ** 2
    assert not b1.any() and not b2.any() and not b3.any()
    m2 = O.Mlp(784, 512, 512, 2, seed=12)
    assert not np.array_equal(m.params, m2.params)


def test_adam_first_step_and_descent(oracle_lib):
    O = oracle_lib
    X, T, m = _small(O)
    p0 = m.params.copy()
    loss0, g = m.loss_grad(X, T, bf16_ops=False)
    m.adam(g, lr=1e-3)
    # bias-corrected first step: lr * g / (|g| + eps), i.e. lr * sign(g) where g != 0
    step = p0.astype(np.float64) - m.params.astype(np.float64)
    nz = np.abs(g) > 1e-4
    np.testing.assert_allclose(step[nz], 1e-3 * np.sign(g[nz]), rtol=1e-3, atol=1e-7)
    for _ in range(200):
        _, g = m.loss_grad(X, T, bf16_ops=False)
        m.adam(g, lr=1e-2)
    loss1, _ = m.loss_grad(X, T, bf16_ops=False)
    assert loss1 < 0.5 * loss0
