"""Pins of the oracle's step-selector network.

Gradients against central finite differences of the loss (away from the
ReLU kinks), the asymmetric weight of the loss on hand-computed cases, and
Adam against its closed form on a quadratic.
"""
import numpy as np
import pytest

from oracle import mlp


def test_forward_shapes_and_relu():
    p = mlp.init_params(16, seed=1)
    x = np.random.default_rng(0).standard_normal((5, 8))
    o, (xx, z1, h1, z2, h2) = mlp.forward(p, x)
    assert o.shape == (5, 2) and h1.shape == (5, 16)
    assert np.all(h1 >= 0) and np.array_equal(h1, np.where(z1 > 0, z1, 0))
    # a hand-built network: identity-like first layer, sums in the second
    q = {"W1": np.eye(4, 8), "b1": np.array([0.0, -1.0, 0.0, 0.0]),
         "W2": np.ones((4, 4)), "b2": np.zeros(4),
         "W3": np.array([[1.0, 0, 0, 0], [0, 0, 0, 2.0]]), "b3": np.array([0.5, -0.5])}
    xin = np.array([[1.0, 0.5, -2.0, 3.0, 9, 9, 9, 9]])
    o1, _ = mlp.forward(q, xin)
    s = max(1.0, 0) + max(0.5 - 1.0, 0) + max(-2.0, 0) + max(3.0, 0)
    assert np.allclose(o1, [[s + 0.5, 2 * s - 0.5]])


def test_loss_asymmetric_weight():
    o = np.array([[1.0, 5.0]])
    t = np.array([[3.0, 4.0]])
    # first output under-predicts by 2 (weight kappa), second over-predicts by 1
    assert mlp.loss(o, t, kappa=4.0) == pytest.approx(0.5 * (4 * 4 + 1))
    assert mlp.loss(t, t) == 0.0


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    p = mlp.init_params(12, seed=2)
    x = rng.standard_normal((7, 8))
    t = rng.standard_normal((7, 2))
    o, cache = mlp.forward(p, x)
    g = mlp.backward(p, cache, o, t, kappa=3.0)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss(mlp.forward(p, x)[0], t, 3.0)
            flat[idx] = old - eps
            lm = mlp.loss(mlp.forward(p, x)[0], t, 3.0)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert g[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (k, idx)


def test_adam_closed_form_first_steps():
    """With a constant gradient g, the bias-corrected moments are exactly g
    and g^2, so each step moves by lr * g / (|g| + eps)."""
    p = {"a": np.array([1.0, -2.0])}
    g = {"a": np.array([0.3, -4.0])}
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    for step in range(1, 4):
        before = p["a"].copy()
        mlp.adam_step(p, g, m, v, step, lr=0.01)
        assert np.allclose(p["a"] - before, -0.01 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-9)


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((64, 8))
    t = np.stack([x[:, 0] * 2 + 1, np.abs(x[:, 1])], axis=1)
    p = mlp.init_params(16, seed=4)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    l0 = mlp.loss(mlp.forward(p, x)[0], t)
    for step in range(1, 301):
        o, c = mlp.forward(p, x)
        mlp.adam_step(p, mlp.backward(p, c, o, t), m, v, step, lr=1e-2)
    assert mlp.loss(mlp.forward(p, x)[0], t) < 0.05 * l0
