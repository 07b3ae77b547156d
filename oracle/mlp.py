"""Step-selector network in float64 numpy: forward, loss, backward, Adam.

Test infrastructure only (see the package docstring).

The network maps a feature vector x (8 values) to two outputs through two
hidden layers of width H with ReLU:

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  o = W3 h2 + b3

Weights are row-major: W1 is H x 8, W2 is H x H, W3 is 2 x H.  The loss is
an asymmetric squared error: for target t and output o,

    L = 1/(2n) sum over samples and outputs of  w * (o - t)^2,
    w = kappa where o < t (under-prediction), else 1,

so predicting too few products (which costs a fallback) is penalised
kappa times more than predicting too many.  Adam with the textbook
bias-corrected moments (Kingma & Ba) updates the parameters.
"""
from __future__ import annotations

import numpy as np

N_IN = 8
N_OUT = 2


def init_params(hidden: int = 64, seed: int = 0) -> dict:
    """He-uniform weights (bound sqrt(6/fan_in)), zero biases, float64."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    shapes = {"W1": (hidden, N_IN), "W2": (hidden, hidden), "W3": (N_OUT, hidden)}
    p = {}
    for name, (fo, fi) in shapes.items():
        bound = np.sqrt(6.0 / fi)
        p[name] = rng.uniform(-bound, bound, size=(fo, fi))
    p["b1"] = np.zeros(hidden)
    p["b2"] = np.zeros(hidden)
    p["b3"] = np.zeros(N_OUT)
    return p


def forward(p: dict, x: np.ndarray):
    """x: n x 8.  Returns (o, cache) with o: n x 2."""
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (x, z1, h1, z2, h2)


def loss(o: np.ndarray, t: np.ndarray, kappa: float = 4.0) -> float:
    w = np.where(o < t, kappa, 1.0)
    return float(0.5 * np.sum(w * (o - t) ** 2) / o.shape[0])


def backward(p: dict, cache, o: np.ndarray, t: np.ndarray, kappa: float = 4.0) -> dict:
    """Gradients of `loss` with respect to every parameter."""
    x, z1, h1, z2, h2 = cache
    n = o.shape[0]
    w = np.where(o < t, kappa, 1.0)
    do = w * (o - t) / n
    g = {"W3": do.T @ h2, "b3": do.sum(axis=0)}
    dh2 = do @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update in place; `step` counts from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
