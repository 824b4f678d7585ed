"""FP64 numpy twin of the cost-model MLP (test infrastructure only).

Network: x -> Linear(h) -> ReLU -> Linear(h) -> ReLU -> Linear(1); loss = mean over the batch of (y - t)^2;
optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction. Flat parameter layout:
W1[h][nin], b1[h], W2[h][h], b2[h], W3[h], b3. Pinned by tests/test_mlp_oracle.py (central finite differences
of the loss, the closed form of Adam's first step, hand-computed tiny networks).
"""
from __future__ import annotations

import numpy as np


def sizes(nin: int, h: int) -> int:
    return h * nin + h + h * h + h + h + 1


def unpack(p: np.ndarray, nin: int, h: int):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * nin].reshape(h, nin); o += h * nin
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h]; o += h
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p, X, nin, h):
    W1, b1, W2, b2, W3, b3 = unpack(p, nin, h)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2.T + b2
    A2 = np.maximum(Z2, 0.0)
    Y = A2 @ W3 + b3
    return Y, (X, Z1, A1, Z2, A2)


def loss(p, X, T, nin, h) -> float:
    Y, _ = forward(p, X, nin, h)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(p, X, T, nin, h):
    """Analytic gradient of the mean squared error (back-propagation), same flat layout as p."""
    W1, b1, W2, b2, W3, b3 = unpack(p, nin, h)
    Y, (X, Z1, A1, Z2, A2) = forward(p, X, nin, h)
    B = X.shape[0]
    dY = 2.0 * (Y - np.asarray(T, dtype=np.float64)) / B          # (B,)
    gW3 = A2.T @ dY                                               # (h,)
    gb3 = dY.sum()
    dZ2 = np.outer(dY, W3) * (Z2 > 0)                             # (B, h)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]]), float(np.mean((Y - T) ** 2))


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
