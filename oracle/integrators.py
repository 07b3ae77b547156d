"""phi_k(tau A) v by Newton interpolation at Leja points, and the exponential
Euler step.

Test infrastructure only (see the package docstring).

Sec. II-C: with an a-priori bound [a, b] of the field of values of A,
polynomial interpolation reduces phi_k(tau A) v to repeated products
(alpha A + beta I) x (eq. (3)).  Sec. III-C names interpolation at Leja
points.  The steps, in the order this module performs them:

1. Interval: [a, b] from Gershgorin (``operators.gershgorin_interval``) unless
   the caller supplies one.  Centre ``c = (a + b)/2``, quarter-width
   ``gamma = (b - a)/4``, so that ``(A - cI)/gamma`` has its spectrum in
   [-2, 2].
2. Substeps: ``s = max(1, ceil(tau (b - a) / l_max))`` and ``delta = tau/s``.
3. Divided differences ``d_j`` of ``x -> phi_k(delta (c + gamma x))`` at the
   Leja points ``xi_0..xi_{m_max}`` of [-2, 2] (``leja.divided_differences``).
4. Newton form applied to a vector r: ``w_0 = r``, ``p = d_0 w_0`` and for
   ``j = 0, 1, ...``::

       w_{j+1} = (alpha A + beta_j I) w_j,  alpha = 1/gamma,
                                            beta_j = -(c/gamma + xi_j)
       p      += d_{j+1} w_{j+1}

   i.e. ``w_{j+1} = ((A - cI)/gamma - xi_j I) w_j``; every step is one
   product of the form of eq. (3).
5. Stop test (the paper fixes only that a tolerance controls the number of
   products, Tables IV and V): with ``t_j = |d_j| ||w_j||_2``, stop after the
   first step ``m = j + 1 >= 2`` with ``t_{m-1} + t_m <= tol ||p||_2``.
   If ``m_max`` steps pass without stopping, the substep count doubles and the
   whole evaluation restarts (at most ``max_retries`` times).
6. Substeps of phi_1: ``y(t) = t phi_1(tA) v`` solves ``y' = A y + v``,
   ``y(0) = 0``, and ``e^{dA} = I + dA phi_1(dA)``, hence
   ``y_{l+1} = y_l + delta phi_1(delta A)(A y_l + v)`` and
   ``phi_1(tau A) v = y_s / tau``.  For phi_0, ``y_{l+1} = e^{delta A} y_l``.
   For k >= 2, ``y(t) = t^k phi_k(tA) v`` solves ``y' = A y + t^(k-1)/(k-1)! v``,
   ``y(0) = 0``; by variation of constants one substep from ``t = l delta`` is
   ``y_{l+1} = e^{X} y_l + sum_{j=1..k} delta^j t^(k-j)/(k-j)! phi_j(X) v``
   with ``X = delta A``.  Any sum ``sum_{j=0..k} phi_j(X) b_j`` equals
   ``sum_{j<k} w_j / j! + phi_k(X) w_k`` with ``w_0 = b_0``,
   ``w_j = X w_{j-1} + b_j`` (from ``phi_j(X) = I/j! + X phi_{j+1}(X)``), so a
   substep costs k products plus one Newton loop for phi_k.  The module
   carries ``z_l = y_l / tau^k``, for which ``b_0 = z_l`` and
   ``b_j = s^-j (l/s)^(k-j)/(k-j)! v``, and returns ``z_s``.
7. Exponential Euler, eq. (2), for ``u' = A u + g(u)`` (the paper writes
   ``u' + A u = g`` with A having large negative eigenvalues; with A the
   discrete Laplacian itself, whose eigenvalues are negative, the sign of A
   flips and eq. (2) reads ``u_{n+1} = e^{tau A} u_n + tau phi_1(tau A) g(u_n)``).
   Using ``e^{tau A} = I + tau A phi_1(tau A)`` this equals
   ``u_n + tau phi_1(tau A)(A u_n + g(u_n))``; with substeps,
   ``y_0 = u_n``, ``y_{l+1} = y_l + delta phi_1(delta A)(A y_l + g(u_n))``,
   ``u_{n+1} = y_s``.
9. Complex operators (Sec. II-C allows K = C; the spin system of Sec. III-D
   solves psi' = -i H psi with H Hermitian, stored in CSR):
   ``skew_phi_action`` gives ``phi_k(-i tau H) v``, k = 0 or 1, by the same
   Newton recurrence (real alpha, beta_j applied to H) with the complex
   divided differences of ``x -> phi_k(-i delta (c + gamma x))``, [a, b] the
   Gershgorin interval of H, and the substep rules of steps 2 and 6 with
   A = -i H.
8. The second-order exponential Runge-Kutta method with c_2 = 1 (one of the
   higher-order methods the paper points to, Sec. II-C; Hochbruck and
   Ostermann's review): the exponential Euler step gives the stage U, then
   ``u_{n+1} = U + tau phi_2(tau A)(g(U) - g(u_n))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import leja
from .operators import gershgorin_interval


@dataclass(frozen=True)
class LejaParams:
    l_max: float = 100.0     # largest delta*(b-a) per substep
    m_max: int = 100         # largest number of Newton steps per substep
    max_retries: int = 4     # substep doublings after a non-converged substep


@dataclass
class Stats:
    substeps: int = 0
    newton_steps: int = 0    # products inside the Newton loops
    matvecs: int = 0         # all products with A (Newton + start vectors)
    degrees: list = field(default_factory=list)
    err_est: float = 0.0     # largest (t_{m-1} + t_m)/||p|| over the substeps
    converged: bool = True
    retries: int = 0
    interval: tuple = (0.0, 0.0)


def substep_count(tau: float, a: float, b: float, l_max: float) -> int:
    """Step 2: ``s = max(1, ceil(tau (b - a) / l_max))``."""
    return max(1, int(math.ceil(tau * (b - a) / l_max)))


def newton_leja(A, r: np.ndarray, d: np.ndarray, xi: np.ndarray, c: float,
                gamma: float, tol: float, m_max: int):
    """Steps 4-5 on one vector.  Returns ``(p, m, err, converged)`` where
    ``m`` is the number of products and ``err = (t_{m-1} + t_m)/||p||``."""
    alpha = 1.0 / gamma
    # complex when the operator, the vector or the coefficients are (K = C)
    w = np.array(r, dtype=np.result_type(r, d, A.dtype, np.float64), copy=True)
    p = d[0] * w
    t_prev = abs(d[0]) * np.linalg.norm(w)
    err = math.inf
    for j in range(m_max):
        beta = -(c / gamma + xi[j])
        w = alpha * (A @ w) + beta * w
        p = p + d[j + 1] * w
        t = abs(d[j + 1]) * np.linalg.norm(w)
        pn = np.linalg.norm(p)
        m = j + 1
        err = (t_prev + t) / pn if pn > 0 else (0.0 if t_prev + t == 0 else math.inf)
        if m >= 2 and t_prev + t <= tol * pn:
            return p, m, err, True
        t_prev = t
    return p, m_max, err, False


def _interval(A, interval):
    if interval is not None:
        a, b = float(interval[0]), float(interval[1])
    else:
        a, b = gershgorin_interval(A)
    if not a < b:
        raise ValueError("degenerate interval: need a < b")
    return a, b


def phi_action(A, k: int, tau: float, v: np.ndarray, tol: float,
               interval=None, params: LejaParams = LejaParams()):
    """``phi_k(tau A) v`` (steps 1-6).  Returns ``(y, Stats)``."""
    if k < 0:
        raise ValueError("k must be non-negative")
    v = np.asarray(v, dtype=np.float64)
    a, b = _interval(A, interval)
    c, gamma = 0.5 * (a + b), 0.25 * (b - a)
    s = substep_count(tau, a, b, params.l_max)
    xi = leja.leja_points(params.m_max + 1)
    st = Stats(interval=(a, b))
    for attempt in range(params.max_retries + 1):
        delta = tau / s
        d = leja.divided_differences(k, delta, c, gamma, xi)
        st = Stats(interval=(a, b), substeps=s, retries=attempt)
        ok = True
        if k == 0:
            y = v.copy()
            for _ in range(s):
                y, m, err, conv = newton_leja(A, y, d, xi, c, gamma, tol, params.m_max)
                st.newton_steps += m
                st.degrees.append(m)
                st.err_est = max(st.err_est, err)
                ok &= conv
            out = y
        elif k == 1:
            y = np.zeros_like(v)
            for l in range(s):
                r = v if l == 0 else (A @ y) + v
                if l > 0:
                    st.matvecs += 1
                p, m, err, conv = newton_leja(A, r, d, xi, c, gamma, tol, params.m_max)
                st.newton_steps += m
                st.degrees.append(m)
                st.err_est = max(st.err_est, err)
                ok &= conv
                y = y + delta * p
            out = y / tau
        elif s == 1:
            out, m, err, conv = newton_leja(A, v, d, xi, c, gamma, tol, params.m_max)
            st.newton_steps += m
            st.degrees.append(m)
            st.err_est = err
            ok = conv
        else:
            # k >= 2 with substeps (step 6): z_l = y(l delta) / tau^k
            z = np.zeros_like(v)
            for l in range(s):
                w = z.copy()                  # w_0 = b_0 = z_l
                acc = w.copy()                # sum_{j<k} w_j / j!
                for j in range(1, k + 1):
                    b_j = (s ** -j) * (l / s) ** (k - j) / math.factorial(k - j) * v
                    if np.any(w):
                        w = delta * (A @ w) + b_j
                        st.matvecs += 1
                    else:
                        w = b_j
                    if j < k:
                        acc = acc + w / math.factorial(j)
                p, m, err, conv = newton_leja(A, w, d, xi, c, gamma, tol, params.m_max)
                st.newton_steps += m
                st.degrees.append(m)
                st.err_est = max(st.err_est, err)
                ok &= conv
                z = acc + p
            out = z
        st.matvecs += st.newton_steps
        st.converged = ok
        if ok:
            return out, st
        s *= 2
    return out, st


def cubic(u: np.ndarray) -> np.ndarray:
    """The reaction term ``g(u) = u - u^3``."""
    return u - u * u * u


def combustion(u: np.ndarray) -> np.ndarray:
    """The combustion nonlinearity of Sec. III-C, computed pointwise:
    ``g(u) = (2 - u)/4 exp(20 (1 - 1/u))`` (g(0) = 0 as the limit from above,
    which the float64 evaluation reaches through 1/0 = inf)."""
    u = np.asarray(u, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return 0.25 * (2.0 - u) * np.exp(20.0 * (1.0 - 1.0 / u))


def expeuler_step(A, tau: float, u: np.ndarray, tol: float, g=cubic,
                  interval=None, params: LejaParams = LejaParams(), forcing=None):
    """One exponential Euler step (step 7).  Returns ``(u_next, Stats)``.
    ``forcing``: a constant vector added to g(u) (the boundary term b_f of
    inhomogeneous Dirichlet data, for which the right-hand side is
    ``A_0 u + b_f + g(u)``)."""
    u = np.asarray(u, dtype=np.float64)
    a, b = _interval(A, interval)
    c, gamma = 0.5 * (a + b), 0.25 * (b - a)
    s = substep_count(tau, a, b, params.l_max)
    xi = leja.leja_points(params.m_max + 1)
    gn = g(u)
    if forcing is not None:
        gn = gn + np.asarray(forcing, dtype=np.float64)
    st = Stats(interval=(a, b))
    for attempt in range(params.max_retries + 1):
        delta = tau / s
        d = leja.divided_differences(1, delta, c, gamma, xi)
        st = Stats(interval=(a, b), substeps=s, retries=attempt)
        ok = True
        y = u.copy()
        for _ in range(s):
            r = (A @ y) + gn
            st.matvecs += 1
            p, m, err, conv = newton_leja(A, r, d, xi, c, gamma, tol, params.m_max)
            st.newton_steps += m
            st.degrees.append(m)
            st.err_est = max(st.err_est, err)
            ok &= conv
            y = y + delta * p
        st.matvecs += st.newton_steps
        st.converged = ok
        if ok:
            return y, st
        s *= 2
    return y, st


def exprk2_step(A, tau: float, u: np.ndarray, tol: float, g=cubic,
                interval=None, params: LejaParams = LejaParams(), forcing=None):
    """One step of the second-order exponential Runge-Kutta method (step 8):
    ``U = u + tau phi_1(tau A)(A u + g(u))`` (the exponential Euler step),
    then ``u_{n+1} = U + tau phi_2(tau A)(g(U) - g(u))``.  Returns
    ``(u_next, (Stats of the stage, Stats of the phi_2 action))``."""
    u = np.asarray(u, dtype=np.float64)
    U, st1 = expeuler_step(A, tau, u, tol, g, interval, params, forcing)
    p2, st2 = phi_action(A, 2, tau, g(U) - g(u), tol, interval, params)
    return U + tau * p2, (st1, st2)


def skew_phi_action(H, k: int, tau: float, v: np.ndarray, tol: float,
                    interval=None, params: LejaParams = LejaParams()):
    """``phi_k(-i tau H) v`` for Hermitian H (step 9), k = 0 or 1.
    Returns ``(y, Stats)``; y is complex128."""
    if k not in (0, 1):
        raise ValueError("k must be 0 or 1")
    v = np.asarray(v, dtype=np.complex128)
    a, b = _interval(H, interval)
    c, gamma = 0.5 * (a + b), 0.25 * (b - a)
    s = substep_count(tau, a, b, params.l_max)
    xi = leja.leja_points(params.m_max + 1)
    st = Stats(interval=(a, b))
    for attempt in range(params.max_retries + 1):
        delta = tau / s
        d = leja.divided_differences_skew(k, delta, c, gamma, xi)
        st = Stats(interval=(a, b), substeps=s, retries=attempt)
        ok = True
        y = v.copy() if k == 0 else np.zeros_like(v)
        for l in range(s):
            if k == 0:
                r = y
            else:
                # y(t) = t phi_1(-i t H) v solves y' = -i H y + v
                r = v if l == 0 else -1j * (H @ y) + v
                if l > 0:
                    st.matvecs += 1
            p, m, err, conv = newton_leja(H, r, d, xi, c, gamma, tol, params.m_max)
            st.newton_steps += m
            st.degrees.append(m)
            st.err_est = max(st.err_est, err)
            ok &= conv
            y = p if k == 0 else y + delta * p
        st.matvecs += st.newton_steps
        st.converged = ok
        if ok:
            return (y if k == 0 else y / tau), st
        s *= 2
    return (y if k == 0 else y / tau), st
