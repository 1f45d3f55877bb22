"""Float64 reference of the cost model's MLP (in -> H -> H -> 1, ReLU) and of
its mean-squared-error gradient, written out with numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring). Parameter layout: one
flat array W1[H][in], b1[H], W2[H][H], b2[H], W3[H], b3[1]."""
from __future__ import annotations

import numpy as np


def unpack(p: np.ndarray, n_in: int, h: int):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + h * n_in].reshape(h, n_in); o += h * n_in
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h]; o += h
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(p, n_in, h, x):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h)
    x = np.asarray(x, np.float64)
    z1 = x @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ W3 + b3[0]
    return y, (x, z1, a1, z2, a2)


def loss(p, n_in, h, x, t):
    y, _ = forward(p, n_in, h, x)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p, n_in, h, x, t):
    """d loss / d p by the chain rule, same layout as p."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h)
    y, (x, z1, a1, z2, a2) = forward(p, n_in, h, x)
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    dW3 = a2.T @ dy
    db3 = np.array([dy.sum()])
    d2 = np.outer(dy, W3) * (z2 > 0)
    dW2 = d2.T @ a1
    db2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    dW1 = d1.T @ x
    db1 = d1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, db3])


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
