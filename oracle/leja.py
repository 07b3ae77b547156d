"""Leja points on [-2, 2] and divided differences of the phi functions.

Test infrastructure only (see the package docstring).

Sec. III-C evaluates the matrix functions by polynomial interpolation at Leja
points.  The paper names the method and leaves its details to the cited
review; the definitions used here are the standard ones:

* Leja points of the reference interval [-2, 2]: ``xi_0 = 2`` and
  ``xi_k`` maximises ``prod_{j<k} |xi - xi_j|`` over [-2, 2].  When two
  candidates give the same product (to a relative 1e-10), the larger one is
  taken.  The maximisation is exact, not over a grid: between two
  consecutive earlier points the product is smooth and positive and its
  logarithmic derivative ``sum_j 1/(xi - xi_j)`` falls strictly from +inf to
  -inf, so each gap holds exactly one local maximum, found by bisection on
  that derivative.
* phi functions: ``phi_0(z) = e^z`` and ``phi_k(z) = sum_{i>=0} z^i/(i+k)!``,
  i.e. ``phi_{k+1}(z) = (phi_k(z) - 1/k!)/z``; ``phi_1`` is the entire
  function of the exponential Euler method, eq. (2).
* Newton divided differences ``f[xi_0, ..., xi_j]`` by the textbook
  recurrence, carried out in 80-digit mpmath arithmetic and rounded to
  float64 at the end.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np

MP_DPS = 80
TIE_RTOL = 1e-10


@functools.lru_cache(maxsize=None)
def _leja_table(count: int) -> tuple:
    pts = [2.0, -2.0]
    while len(pts) < count:
        x = np.asarray(pts)
        s = np.sort(x)
        lo = s[:-1].copy()
        hi = s[1:].copy()
        # bisection on the logarithmic derivative, all gaps at once
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            done = (mid <= lo) | (mid >= hi)
            if np.all(done):
                break
            deriv = np.sum(1.0 / (mid[:, None] - x[None, :]), axis=1)
            live = ~done
            lo = np.where(live & (deriv >= 0.0), mid, lo)
            hi = np.where(live & (deriv <= 0.0), mid, hi)
        cand = 0.5 * (lo + hi)
        logprod = np.sum(np.log(np.abs(cand[:, None] - x[None, :])), axis=1)
        best = int(np.argmax(logprod))
        for i in range(len(cand)):
            if abs(logprod[i] - logprod[best]) <= TIE_RTOL * max(1.0, abs(logprod[best])) \
                    and cand[i] > cand[best]:
                best = i
        pts.append(float(cand[best]))
    return tuple(pts[:count])


def leja_points(count: int) -> np.ndarray:
    """The first ``count`` Leja points of [-2, 2] (float64)."""
    if count < 1:
        raise ValueError("count must be positive")
    if count == 1:
        return np.array([2.0])
    return np.array(_leja_table(int(count)), dtype=np.float64)


def phi_mp(k: int, z):
    """phi_k(z) in mpmath arithmetic (``z`` an mpf)."""
    z = mpmath.mpf(z)
    if k == 0:
        return mpmath.exp(z)
    if abs(z) < mpmath.mpf("0.5"):
        # power series sum_i z^i/(i+k)!; terms shrink by |z|/(i+k+1) <= 1/4
        term = mpmath.mpf(1) / mpmath.factorial(k)
        total = term
        i = 0
        while abs(term) > mpmath.mpf(10) ** (-(MP_DPS + 5)):
            i += 1
            term = term * z / (i + k)
            total += term
        return total
    val = mpmath.expm1(z) / z
    for j in range(1, k):
        val = (val - mpmath.mpf(1) / mpmath.factorial(j)) / z
    return val


def phi(k: int, z: float) -> float:
    """phi_k(z) rounded to float64."""
    with mpmath.workdps(MP_DPS):
        return float(phi_mp(k, z))


def divided_differences(k: int, delta: float, c: float, gamma: float,
                        xi: np.ndarray) -> np.ndarray:
    """Divided differences of ``f(x) = phi_k(delta * (c + gamma * x))`` at the
    nodes ``xi`` (float64 in, float64 out; computed at 80 digits).

    This is the function of the reference variable x in [-2, 2] whose
    interpolant, evaluated at ``(A - cI)/gamma``, approximates
    ``phi_k(delta A)`` (Sec. III-C).
    """
    with mpmath.workdps(MP_DPS):
        x = [mpmath.mpf(float(v)) for v in xi]
        dl, cc, gg = mpmath.mpf(float(delta)), mpmath.mpf(float(c)), mpmath.mpf(float(gamma))
        d = dd_recurrence([phi_mp(k, dl * (cc + gg * t)) for t in x], x)
        return np.array([float(v) for v in d], dtype=np.float64)


def phi_mpc(k: int, z):
    """phi_k(z) in mpmath arithmetic for complex ``z`` (an mpc)."""
    z = mpmath.mpc(z)
    if k == 0:
        return mpmath.exp(z)
    if abs(z) < mpmath.mpf("0.5"):
        term = mpmath.mpf(1) / mpmath.factorial(k)
        total = term
        i = 0
        while abs(term) > mpmath.mpf(10) ** (-(MP_DPS + 5)):
            i += 1
            term = term * z / (i + k)
            total += term
        return total
    val = mpmath.expm1(z) / z
    for j in range(1, k):
        val = (val - mpmath.mpf(1) / mpmath.factorial(j)) / z
    return val


def divided_differences_skew(k: int, delta: float, c: float, gamma: float,
                             xi: np.ndarray) -> np.ndarray:
    """Divided differences of ``f(x) = phi_k(-i delta (c + gamma x))`` at the
    real nodes ``xi`` (complex128 out; 80 digits).  With H Hermitian and its
    spectrum in [a, b] = [c - 2 gamma, c + 2 gamma], ``(H - cI)/gamma`` has
    its spectrum in [-2, 2] and the interpolant evaluated there approximates
    ``phi_k(-i delta H)``: Sec. II-C's products (alpha A + beta I) x with
    K = C, where alpha and beta stay real and the coefficients are complex."""
    with mpmath.workdps(MP_DPS):
        x = [mpmath.mpf(float(v)) for v in xi]
        dl, cc, gg = mpmath.mpf(float(delta)), mpmath.mpf(float(c)), mpmath.mpf(float(gamma))
        d = dd_recurrence([phi_mpc(k, mpmath.mpc(0, -1) * dl * (cc + gg * t)) for t in x], x)
        return np.array([complex(v) for v in d], dtype=np.complex128)


def dd_recurrence(values, nodes):
    """Newton divided differences ``f[x_0..x_j]``, ``j = 0..m-1``, from the
    values ``f(x_i)`` by the textbook in-place recurrence
    ``d_i <- (d_i - d_{i-1}) / (x_i - x_{i-j})`` for ``j = 1..m-1`` and
    ``i = m-1 .. j``.  Works on any numbers that support the arithmetic
    (mpmath mpf inside ``divided_differences``)."""
    d = list(values)
    x = list(nodes)
    m = len(x)
    if len(d) != m:
        raise ValueError("values and nodes differ in length")
    for j in range(1, m):
        for i in range(m - 1, j - 1, -1):
            d[i] = (d[i] - d[i - 1]) / (x[i] - x[i - j])
    return d


def newton_eval(d: np.ndarray, xi: np.ndarray, x) -> np.ndarray:
    """Evaluate the Newton-form polynomial ``sum_j d_j prod_{i<j} (x - xi_i)``
    at scalar or array ``x`` (float64)."""
    x = np.asarray(x, dtype=np.float64)
    total = np.zeros_like(x)
    basis = np.ones_like(x)
    for j in range(len(d)):
        total = total + d[j] * basis
        basis = basis * (x - xi[j])
    return total


__all__ = ["leja_points", "phi", "phi_mp", "phi_mpc", "divided_differences",
           "divided_differences_skew", "dd_recurrence", "newton_eval",
           "MP_DPS", "TIE_RTOL"]
