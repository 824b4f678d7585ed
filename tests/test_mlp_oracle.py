"""Pins of the FP64 MLP twin (CPU): finite differences, Adam's closed-form first step, a hand-computed net."""
import numpy as np
import pytest

from oracle import mlp


def _setup(seed, nin=7, h=5, B=9):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal(mlp.sizes(nin, h)) * 0.5
    X = rng.standard_normal((B, nin))
    T = rng.standard_normal(B)
    return p, X, T, nin, h


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p, X, T, nin, h = _setup(seed)
    g, _ = mlp.grad(p, X, T, nin, h)
    eps = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        d = np.zeros_like(p)
        d[i] = eps
        num[i] = (mlp.loss(p + d, X, T, nin, h) - mlp.loss(p - d, X, T, nin, h)) / (2 * eps)
    assert np.max(np.abs(g - num)) < 1e-7 * max(1.0, np.max(np.abs(num)))


def test_hand_computed_tiny_network():
    # nin = 1, h = 1: y = w3 relu(w2 relu(w1 x + b1) + b2) + b3
    nin, h = 1, 1
    p = np.array([2.0, 0.5, -1.5, 4.0, 3.0, 0.25])  # W1, b1, W2, b2, W3, b3
    X = np.array([[1.0], [-1.0]])
    # x = 1: z1 = 2.5, a1 = 2.5, z2 = 0.25, a2 = 0.25, y = 1.0
    # x = -1: z1 = -1.5, a1 = 0, z2 = 4, a2 = 4, y = 12.25
    Y, _ = mlp.forward(p, X, nin, h)
    assert np.allclose(Y, [1.0, 12.25])
    T = np.array([0.0, 12.0])
    # loss = (1 + 0.0625) / 2
    assert mlp.loss(p, X, T, nin, h) == pytest.approx(0.53125)
    g, _ = mlp.grad(p, X, T, nin, h)
    # dY = (1, 0.25); gW3 = 1*0.25 + 0.25*4 = 1.25; gb3 = 1.25
    assert g[4] == pytest.approx(1.25) and g[5] == pytest.approx(1.25)


def test_adam_first_step_closed_form():
    rng = np.random.Generator(np.random.PCG64(5))
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    # after bias correction m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))


def test_planted_gradient_mistake_is_caught():
    p, X, T, nin, h = _setup(3)
    g, _ = mlp.grad(p, X, T, nin, h)
    bad = g.copy()
    bad[: h * nin] *= 0.5  # a dropped factor in the first layer's gradient
    eps = 1e-6
    i = 3
    d = np.zeros_like(p)
    d[i] = eps
    num = (mlp.loss(p + d, X, T, nin, h) - mlp.loss(p - d, X, T, nin, h)) / (2 * eps)
    assert abs(g[i] - num) < 1e-7 and abs(bad[i] - num) > 1e-4 * max(abs(num), 1e-3)
