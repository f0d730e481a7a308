"""Pins of the selector network's FP64 reference (oracle/mlp.py)."""
import numpy as np

from oracle import mlp


def _setup(seed=0, n_in=5, hidden=7, B=9):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.param_count(n_in, hidden)) * 0.5
    X = rng.standard_normal((B, n_in))
    y = rng.standard_normal(B)
    return p, X, y, n_in, hidden


def test_gradient_matches_central_differences():
    p, X, y, n_in, hidden = _setup()
    L, g = mlp.loss_grad(p, X, y, n_in, hidden)
    assert abs(L - mlp.loss(p, X, y, n_in, hidden)) < 1e-15
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss(p + e, X, y, n_in, hidden) - mlp.loss(p - e, X, y, n_in, hidden)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_linear_regime_equals_matrix_product():
    # large positive biases keep every ReLU active: f = W3 (W2 (W1 x + b1) + b2) + b3
    p, X, y, n_in, hidden = _setup(1)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, hidden)
    q = p.copy()
    o = hidden * n_in
    q[o:o + hidden] = 100.0
    o2 = o + hidden + hidden * hidden
    q[o2:o2 + hidden] = 1000.0
    W1, b1, W2, b2, W3, b3 = mlp.unpack(q, n_in, hidden)
    f = mlp.forward(q, X, n_in, hidden)
    expect = ((X @ W1.T + b1) @ W2.T + b2) @ W3 + b3
    np.testing.assert_allclose(f, expect, rtol=1e-12)


def test_first_adam_step_is_signed_learning_rate():
    # t = 1: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 1.0, 1.0, 1.0])
    q, m, v = mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(2)
    n_in, hidden = 3, 16
    X = rng.uniform(-1, 1, (256, n_in))
    y = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    p = rng.standard_normal(mlp.param_count(n_in, hidden)) * 0.3
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss(p, X, y, n_in, hidden)
    for t in range(1, 401):
        _, g = mlp.loss_grad(p, X, y, n_in, hidden)
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
    assert mlp.loss(p, X, y, n_in, hidden) < 0.1 * L0
