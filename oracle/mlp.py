"""FP64 reference of the variant-selector network (oracle; test infrastructure only).

A three-layer perceptron in -> H -> H -> 1 with ReLU after the first two
layers, trained on mean squared error with Adam (Kingma and Ba, "Adam: a
method for stochastic optimization", ICLR 2015).  Parameters are one flat
vector in the order W1 (H x in, row-major), b1 (H), W2 (H x H), b2 (H),
W3 (H), b3 (1), the layout the HIP kernels use.

Pinned by: central finite differences of the loss; the closed-form first Adam
step; the linear special case (every ReLU active) against the explicit matrix
product.
"""
from __future__ import annotations

import numpy as np


def param_count(n_in: int, hidden: int) -> int:
    return hidden * n_in + hidden + hidden * hidden + hidden + hidden + 1


def unpack(p, n_in, hidden):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + hidden * n_in].reshape(hidden, n_in); o += hidden * n_in
    b1 = p[o:o + hidden]; o += hidden
    W2 = p[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = p[o:o + hidden]; o += hidden
    W3 = p[o:o + hidden]; o += hidden
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p, X, n_in, hidden, keep=False):
    """Predictions f(X) for a batch X (B x in)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, hidden)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    f = h2 @ W3 + b3
    if keep:
        return f, (X, z1, h1, z2, h2)
    return f


def loss(p, X, y, n_in, hidden):
    f = forward(p, X, n_in, hidden)
    return float(np.mean((f - np.asarray(y, dtype=np.float64)) ** 2))


def loss_grad(p, X, y, n_in, hidden):
    """(loss, gradient) of the mean squared error by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, hidden)
    f, (X, z1, h1, z2, h2) = forward(p, X, n_in, hidden, keep=True)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    df = 2.0 * (f - y) / B                      # dL/df
    gW3 = df @ h2
    gb3 = df.sum()
    dz2 = np.outer(df, W3) * (z2 > 0)           # B x H
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return float(np.mean((f - y) ** 2)), g


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
