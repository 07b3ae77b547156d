"""Pins of the oracle's further workloads of the paper.

* the combustion nonlinearity of Sec. III-C and exponential Euler steps with
  it (closed values, the scalar and diagonal operators in mpmath);
* phi_k(tau A) v for k >= 2 with substeps (sine-mode closed form, dense
  brute force of the augmented matrix);
* the second-order exponential Runge-Kutta step (scalar closed form in
  mpmath, exactness for constant forcing, observed order 2 against a tight
  implicit ODE solve);
* inhomogeneous Dirichlet data (Sec. III-A, Table I): exactness of the
  stencil for quadratic data, second-order consistency, and a second,
  pointwise implementation of the boundary term;
* D(x) times the Laplacian (Sec. III-B, Table II): sine eigenmodes,
  the pointwise implementation, the Gershgorin bound.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.integrate import solve_ivp

import synth
from oracle import integrators as I
from oracle import operators as O


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# combustion nonlinearity (Sec. III-C)
# ---------------------------------------------------------------------------

def test_combustion_values():
    u = np.array([1.0, 2.0, 0.5, 0.0, 1.5, 4.0])
    g = I.combustion(u)
    assert g[0] == 0.25                       # (2-1)/4 e^0
    assert g[1] == 0.0                        # (2-2)/4 ...
    assert g[2] == pytest.approx(0.375 * math.exp(-20.0), rel=1e-15)
    assert g[3] == 0.0                        # limit from above
    assert g[4] == pytest.approx(0.125 * math.exp(20.0 / 3.0), rel=1e-15)
    assert g[5] == pytest.approx(-0.5 * math.exp(15.0), rel=1e-15)
    # monotone decay towards 0 as u -> 0+
    small = I.combustion(np.array([0.2, 0.1, 0.05]))
    assert small[0] > small[1] > small[2] > 0


def _mp_phi(k, z):
    z = mp.mpf(z)
    if z == 0:
        return mp.mpf(1) / mp.factorial(k)
    s = mp.e ** z
    for j in range(k):
        s = (s - mp.mpf(1) / mp.factorial(j)) / z
    return s


def _mp_combustion(u):
    u = mp.mpf(u)
    return (2 - u) / 4 * mp.e ** (20 * (1 - 1 / u))


def test_expeuler_combustion_diagonal_operator_mpmath():
    """A = diag(lambda_i): each component follows the scalar formula
    u1 = e^{tau l} u0 + tau phi_1(tau l) g(u0), evaluated in 50-digit mpmath."""
    mp.mp.dps = 50
    lam = -np.linspace(0.0, 4000.0, 17)
    A = sp.csr_matrix(sp.diags(lam))
    u0 = np.linspace(0.6, 1.9, 17)
    tau = 1e-3
    got, st = I.expeuler_step(A, tau, u0, 1e-13, g=I.combustion, interval=(-4000.0, 0.0))
    want = np.array([float(mp.e ** (tau * l) * u + tau * _mp_phi(1, tau * l) * _mp_combustion(u))
                     for l, u in zip(lam, u0)])
    assert st.converged
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12


# ---------------------------------------------------------------------------
# phi_k, k >= 2, with substeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("length", [60.0, 350.0, 900.0])
def test_phik_substeps_dst_closed_form(k, length):
    shape = (24, 19)
    h = tuple(1.0 / (n + 1) for n in shape)
    A = O.stencil_matrix(shape, h, "dirichlet0")
    a, b = O.gershgorin_interval(A)
    tau = length / (b - a)
    v = synth.uniform_vector(A.shape[0], 5)
    y, st = I.phi_action(A, k, tau, v, 1e-11)
    want = O.dirichlet_box_phi(k, shape, h, tau, v)
    assert st.substeps == max(1, math.ceil(length / 100.0))
    assert relerr(y, want) <= 1e-10


def test_phi2_substeps_variable_coefficient_brute_force():
    """phi_2 of a variable-coefficient Neumann operator with 3 substeps
    against the dense (k+1)-block augmented matrix exponential."""
    n = 7
    shape = (n, n, n)
    h = (1.0 / n,) * 3
    fld = synth.sine_coefficient(n, 0.6).field()
    A = O.stencil_matrix(shape, h, "neumann0", coef=fld)
    a, b = O.gershgorin_interval(A)
    tau = 250.0 / (b - a)
    v = synth.uniform_vector(A.shape[0], 9)
    y, st = I.phi_action(A, 2, tau, v, 1e-12)
    N = A.shape[0]
    M = np.zeros((N + 2, N + 2))
    M[:N, :N] = tau * A.toarray()
    M[:N, N] = v
    M[N, N + 1] = 1.0
    want = sla.expm(M)[:N, N + 1]
    assert st.substeps == 3
    assert relerr(y, want) <= 1e-10


# ---------------------------------------------------------------------------
# second-order exponential Runge-Kutta step
# ---------------------------------------------------------------------------

def test_exprk2_scalar_mpmath():
    mp.mp.dps = 50
    for lam, u0, tau in ((-300.0, 0.7, 1e-2), (-5.0, -1.3, 0.1), (-80.0, 1.2, 4e-2)):
        A = sp.csr_matrix(np.array([[lam]]))
        got, _ = I.exprk2_step(A, tau, np.array([u0]), 1e-14, interval=(2 * lam, 0.0))
        g = lambda u: u - u ** 3
        z = mp.mpf(tau) * lam
        U = mp.e ** z * u0 + tau * _mp_phi(1, z) * g(mp.mpf(u0))
        want = U + tau * _mp_phi(2, z) * (g(U) - g(mp.mpf(u0)))
        assert abs(got[0] - float(want)) <= 1e-13 * abs(float(want))


def test_exprk2_constant_forcing_is_exact():
    """g constant: the phi_2 term vanishes and the step is exact,
    u1 = e^{tau A} u0 + tau phi_1(tau A) b (sine-mode closed form)."""
    shape = (20, 17)
    h = tuple(1.0 / (n + 1) for n in shape)
    A = O.stencil_matrix(shape, h, "dirichlet0")
    u0 = synth.uniform_vector(A.shape[0], 1)
    bvec = synth.uniform_vector(A.shape[0], 2)
    tau = 3e-3
    got, _ = I.exprk2_step(A, tau, u0, 1e-12, g=lambda u: bvec)
    want = O.dirichlet_box_phi(0, shape, h, tau, u0) + tau * O.dirichlet_box_phi(1, shape, h, tau, bvec)
    assert relerr(got, want) <= 1e-10


def test_exprk2_is_second_order_and_euler_first_order():
    """Global error at T against a tight Radau solve: halving tau divides the
    error by about 4 (second-order step) and by about 2 (exponential Euler)."""
    shape = (9, 8)
    h = tuple(1.0 / (n + 1) for n in shape)
    A = O.stencil_matrix(shape, h, "dirichlet0")
    X = O.positions(shape[0], h[0], "dirichlet0")[None, :]
    Y = O.positions(shape[1], h[1], "dirichlet0")[:, None]
    u0 = (1.5 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y) + 0.8 * X * Y).reshape(-1)
    T = 0.08
    ref = solve_ivp(lambda t, u: A @ u + I.cubic(u), (0.0, T), u0, method="Radau",
                    rtol=1e-12, atol=1e-13, jac=A.toarray() if False else None).y[:, -1]
    errs = {"rk2": [], "euler": []}
    for steps in (8, 16, 32):
        tau = T / steps
        u2, ue = u0.copy(), u0.copy()
        for _ in range(steps):
            u2, _ = I.exprk2_step(A, tau, u2, 1e-13)
            ue, _ = I.expeuler_step(A, tau, ue, 1e-13)
        errs["rk2"].append(np.linalg.norm(u2 - ref))
        errs["euler"].append(np.linalg.norm(ue - ref))
    r2 = [errs["rk2"][i] / errs["rk2"][i + 1] for i in range(2)]
    re = [errs["euler"][i] / errs["euler"][i + 1] for i in range(2)]
    assert all(3.3 < r < 4.8 for r in r2), r2
    assert all(1.7 < r < 2.4 for r in re), re
    assert errs["rk2"][-1] < errs["euler"][-1] / 10


# ---------------------------------------------------------------------------
# inhomogeneous Dirichlet data (Sec. III-A, Table I)
# ---------------------------------------------------------------------------

def test_boundary_term_exact_for_quadratic_data():
    """u = z(1-z)xy is linear in x and y and quadratic in z, so the
    seven-point formula is exact for it: with its own values as the
    boundary data, A_0 u + b_f equals the Laplacian -2xy at every node."""
    shape = (11, 9, 13)
    h = tuple(1.0 / (n + 1) for n in shape)
    A0 = O.stencil_matrix(shape, h, "dirichlet0")
    X = O.positions(shape[0], h[0], "dirichlet0")[None, None, :]
    Y = O.positions(shape[1], h[1], "dirichlet0")[None, :, None]
    Z = O.positions(shape[2], h[2], "dirichlet0")[:, None, None]
    u = O.boundary_values("z1mz_xy", X, Y, Z).reshape(-1)
    bf = O.dirichlet_boundary_term(shape, h, "z1mz_xy")
    got = A0 @ u + bf
    want = np.broadcast_to(-2.0 * X * Y, shape[::-1]).reshape(-1)
    assert np.max(np.abs(got - want)) <= 1e-11


def test_boundary_term_second_order_consistency():
    """f = sin(pi z) exp(-xy) on the grid and as boundary data: A_0 f + b_f
    approximates Delta f with an error falling like h^2."""
    errs = []
    for n in (12, 24, 48):
        shape = (n, n, n)
        h = (1.0 / (n + 1),) * 3
        A0 = O.stencil_matrix(shape, h, "dirichlet0")
        X = O.positions(n, h[0], "dirichlet0")[None, None, :]
        Y = O.positions(n, h[1], "dirichlet0")[None, :, None]
        Z = O.positions(n, h[2], "dirichlet0")[:, None, None]
        f = np.broadcast_to(O.boundary_values("sinpiz_expmxy", X, Y, Z), shape).reshape(-1)
        lap = np.broadcast_to(np.sin(np.pi * Z) * np.exp(-X * Y) * (X * X + Y * Y - np.pi ** 2),
                              shape).reshape(-1)
        got = A0 @ f + O.dirichlet_boundary_term(shape, h, "sinpiz_expmxy")
        errs.append(np.max(np.abs(got - lap)))
    assert 3.3 < errs[0] / errs[1] < 4.5 and 3.3 < errs[1] / errs[2] < 4.5, errs


@pytest.mark.parametrize("kind", ["z1mz_xy", "sinpiz_expmxy"])
def test_boundary_term_matches_pointwise_definition(kind):
    shape = (6, 5, 7)
    h = tuple(1.0 / (n + 1) for n in shape)
    A0 = O.stencil_matrix(shape, h, "dirichlet0", coef=1.7)
    u = synth.uniform_vector(A0.shape[0], 3)
    got = A0 @ u + O.dirichlet_boundary_term(shape, h, kind, coef=1.7)
    want = O.apply_at(shape, h, "dirichlet0", u, range(A0.shape[0]), coef=1.7, bdata=kind)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_expeuler_with_boundary_forcing_steady_state():
    """With g = 0 and data f = z(1-z)xy, the state u* = f is not steady
    (A_0 f + b_f = -2xy), but u* solving A_0 u* + b_f = 0 is: an exponential
    Euler step leaves it unchanged."""
    shape = (8, 7, 9)
    h = tuple(1.0 / (n + 1) for n in shape)
    A0 = O.stencil_matrix(shape, h, "dirichlet0")
    bf = O.dirichlet_boundary_term(shape, h, "z1mz_xy")
    from scipy.sparse.linalg import spsolve
    ustar = spsolve(sp.csc_matrix(A0), -bf)
    got, _ = I.expeuler_step(A0, 1e-2, ustar, 1e-12, g=lambda u: np.zeros_like(u), forcing=bf)
    assert relerr(got, ustar) <= 1e-11


# ---------------------------------------------------------------------------
# D(x) times the Laplacian (Sec. III-B, Table II)
# ---------------------------------------------------------------------------

def test_dlap_sine_eigenmode():
    """On a Dirichlet sine mode s (eigenvector of the Laplacian with
    eigenvalue lambda), (D Lap s)_c = D_c lambda s_c at every node."""
    shape = (10, 12, 9)
    h = tuple(1.0 / (n + 1) for n in shape)
    M = O.dlap_matrix(shape, h, "dirichlet0")
    jx, jy, jz = 3, 2, 4
    X = O.positions(shape[0], h[0], "dirichlet0")[None, None, :]
    Y = O.positions(shape[1], h[1], "dirichlet0")[None, :, None]
    Z = O.positions(shape[2], h[2], "dirichlet0")[:, None, None]
    s = (np.sin(jx * np.pi * X) * np.sin(jy * np.pi * Y) * np.sin(jz * np.pi * Z)).reshape(-1)
    lam = sum(-(4.0 / hh ** 2) * np.sin(j * np.pi * hh / 2) ** 2 for j, hh in zip((jx, jy, jz), h))
    D = np.broadcast_to(1.0 / np.sqrt(1.0 + X * X + Y * Y), shape[::-1]).reshape(-1)
    assert np.max(np.abs(M @ s - D * lam * s)) <= 1e-10 * abs(lam)


@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
@pytest.mark.parametrize("shape", [(6, 5, 4), (9, 7)])
def test_dlap_matches_pointwise_definition(bc, shape):
    h = tuple(1.0 / (n + 1) for n in shape)
    M = O.dlap_matrix(shape, h, bc)
    u = synth.uniform_vector(M.shape[0], 8)
    want = O.apply_at(shape, h, bc, u, range(M.shape[0]), dlap=True)
    assert np.max(np.abs(M @ u - want)) <= 1e-12 * np.max(np.abs(want))


def test_dlap_gershgorin_contains_real_spectrum():
    """D Lap is similar to the symmetric D^1/2 Lap D^1/2, so its spectrum is
    real and non-positive, and it lies in the Gershgorin interval."""
    shape = (7, 6, 5)
    h = tuple(1.0 / (n + 1) for n in shape)
    M = O.dlap_matrix(shape, h, "dirichlet0").toarray()
    ev = np.linalg.eigvals(M)
    a, b = O.gershgorin_interval(M)
    assert np.max(np.abs(ev.imag)) <= 1e-9 * np.max(np.abs(ev))
    assert a <= ev.real.min() and ev.real.max() <= b <= 1e-9
