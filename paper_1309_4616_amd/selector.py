"""Learned step selector: features, logging, GPU training, packing.

The network (8 -> H -> H -> 2, float32) predicts, for a Newton loop of the
Leja interpolation, log2 of the substep count and the Newton degree m from
features the plain method has after its first four products (computed the
same way on the device by the selector kernel):

    log10 tau(b-a), tau b, log10 tau, log10 ||r||, log10(t_k / t_0), k = 1..4

with [a, b] the spectral interval, r the start vector and t_k = |d_k| ||w_k||.
Training uses the library's forward, backward and Adam kernels
(expi_mlp_*); this module only marshals arrays and keeps the loop.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from ._binding import check, lib

N_IN, N_OUT = 8, 2


def features(stats: dict, tau: float) -> np.ndarray:
    """Feature vector of one call's first Newton loop from its stats."""
    a, b = stats["interval_a"], stats["interval_b"]
    t = stats["t_first"]
    f = [math.log10(max(tau * (b - a), 1e-300)), tau * b, math.log10(max(tau, 1e-300)),
         math.log10(stats["rnorm"] + 1e-300)]
    for k in range(1, 5):
        f.append(math.log10(t[k] / t[0] + 1e-300) if t[0] > 0 else -300.0)
    return np.array(f, dtype=np.float64)


def targets(stats: dict) -> np.ndarray:
    """(log2 substeps, degree of the first substep) of a converged plain call."""
    return np.array([math.log2(stats["substeps"]), stats["degree_max"]], dtype=np.float64)


def forced_substeps_l_max(length: float, s: int) -> float:
    """l_max that makes the plain method take exactly s substeps when
    tau (b - a) = length: ceil(length / l_max) = ceil(s - 1/2) = s."""
    return length / (s - 0.5)


def substep_candidates(length: float, s_plain: int, sel_l_max: float = 500.0) -> list:
    """Substep counts worth trying for a step of tau (b - a) = length: the
    plain count and those that make each substep about 150 to sel_l_max
    long (never more than the plain count)."""
    c = {s_plain}
    for L in (sel_l_max, 400.0, 300.0, 200.0, 150.0):
        if L <= sel_l_max:
            c.add(max(1, math.ceil(length / L)))
    return sorted(x for x in c if x <= s_plain)


def best_label(run_forced, length: float, s_plain: int, plain_stats: dict,
               sel_l_max: float = 500.0):
    """Label of one logged step: the substep count with the fewest products
    among those that converge (ties to the larger count), and the degree it
    needed.  run_forced(s) runs the step from the same state with exactly s
    substeps and no retries and returns its stats dict, or None if it did
    not converge.  Returns (targets array, {s: matvecs})."""
    tried = {s_plain: plain_stats}
    for s in substep_candidates(length, s_plain, sel_l_max):
        if s not in tried:
            tried[s] = run_forced(s)
    ok = {s: st for s, st in tried.items() if st is not None and st["converged"]}
    best = min(ok, key=lambda s: (ok[s]["matvecs"], -s))
    return (np.array([math.log2(best), ok[best]["degree_max"]], dtype=np.float64),
            {s: (st["matvecs"] if st is not None else None) for s, st in tried.items()})


class Net:
    """Parameters and Adam state on the device; training by library kernels."""

    def __init__(self, hidden: int = 64, seed: int = 0, device="cuda:0"):
        import torch
        self.hidden = hidden
        self.device = torch.device(device)
        self.count = int(lib().expi_mlp_param_count(hidden))
        self.params = torch.as_tensor(init_params(hidden, seed), dtype=torch.float32,
                                      device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def forward(self, x, act=None):
        import torch
        out = torch.empty((x.shape[0], N_OUT), dtype=torch.float32, device=self.device)
        check(lib().expi_mlp_forward(self.hidden, _p(self.params), _p(x), x.shape[0], _p(out),
                                     _p(act) if act is not None else None, _stream(self.device)))
        return out

    def grad(self, x, target, kappa: float = 4.0):
        """(gradient, loss, out) at the current parameters."""
        import torch
        n = x.shape[0]
        act = torch.empty((n, 2 * self.hidden), dtype=torch.float32, device=self.device)
        out = self.forward(x, act)
        g = torch.empty(self.count, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        scratch = torch.empty(int(lib().expi_mlp_scratch_floats(self.hidden, n)),
                              dtype=torch.float32, device=self.device)
        check(lib().expi_mlp_backward(self.hidden, _p(self.params), _p(x), _p(act), _p(out),
                                      _p(target), n, float(kappa), _p(g), _p(loss), _p(scratch),
                                      _stream(self.device)))
        return g, loss, out

    def adam(self, g, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(lib().expi_mlp_adam(self.count, _p(self.params), _p(g), _p(self.m), _p(self.v),
                                  self.step, float(lr), float(beta1), float(beta2), float(eps),
                                  _stream(self.device)))


def init_params(hidden: int, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, packed W1 b1 W2 b2 W3 b3 (float64)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    parts = []
    for fo, fi in ((hidden, N_IN), (hidden, hidden), (N_OUT, hidden)):
        bound = math.sqrt(6.0 / fi)
        parts.append(rng.uniform(-bound, bound, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def train(X: np.ndarray, Y: np.ndarray, hidden: int = 64, epochs: int = 2000, lr: float = 3e-3,
          kappa: float = 4.0, seed: int = 0, device="cuda:0"):
    """Full-batch training on the GPU.  X, Y are raw features/targets; they
    are z-scored here and the statistics are returned for packing.
    Returns (net, norms, loss history)."""
    import torch
    xm, xs = X.mean(axis=0), X.std(axis=0)
    xs = np.where(xs > 1e-12, xs, 1.0)
    ym, ys = Y.mean(axis=0), Y.std(axis=0)
    ys = np.where(ys > 1e-12, ys, 1.0)
    x = torch.as_tensor((X - xm) / xs, dtype=torch.float32, device=device).contiguous()
    t = torch.as_tensor((Y - ym) / ys, dtype=torch.float32, device=device).contiguous()
    net = Net(hidden, seed, device)
    hist = []
    for ep in range(epochs):
        g, loss, _ = net.grad(x, t, kappa)
        net.adam(g, lr=lr)
        if ep % 100 == 0 or ep == epochs - 1:
            hist.append(float(loss.item()))
    return net, {"x_mean": xm, "x_std": xs, "y_mean": ym, "y_std": ys}, hist


def pack(net: Net, norms: dict):
    """Device float buffer for the selector: x_mean, x_std, y_mean, y_std, params."""
    import torch
    head = np.concatenate([norms["x_mean"], norms["x_std"], norms["y_mean"], norms["y_std"]])
    return torch.cat([torch.as_tensor(head, dtype=torch.float32, device=net.device),
                      net.params.detach()]).contiguous()


def predict(net: Net, norms: dict, X: np.ndarray) -> np.ndarray:
    """De-normalised (log2 s, m) predictions for raw features X (host array)."""
    import torch
    x = torch.as_tensor((X - norms["x_mean"]) / norms["x_std"], dtype=torch.float32,
                        device=net.device).contiguous()
    out = net.forward(x).double().cpu().numpy()
    return out * norms["y_std"] + norms["y_mean"]


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
