"""Pins of the oracle's phi_k(tau A) v and exponential Euler step.

Closed forms (sine and cosine eigenbases of the discrete Laplacian), dense
brute force (matrix exponential of the augmented matrix), scipy's
expm_multiply (a different algorithm), a single eigenmode, the scalar
operator, and invariants (mass, symmetry, constants, positivity, linearity).
"""
import math

import numpy as np
import pytest
import scipy.fft as F
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

import synth
from oracle import integrators as I
from oracle import operators as O


def phi_scalar(k, z):
    z = np.asarray(z, dtype=np.float64)
    if k == 0:
        return np.exp(z)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-3
    zs = z[small]
    # series sum_i z^i/(i+k)! to five terms
    ser = np.zeros_like(zs)
    for i in range(6):
        ser += zs ** i / math.factorial(i + k)
    out[small] = ser
    zb = z[~small]
    val = np.expm1(zb) / zb
    for j in range(1, k):
        val = (val - 1.0 / math.factorial(j)) / zb
    out[~small] = val
    return out


def dst_eigvals(shape, h):
    """Eigenvalues of the Dirichlet Laplacian in the DST-I basis, in numpy
    axis order (slowest first)."""
    lam = 0.0
    for d, n in enumerate(shape):
        j = np.arange(1, n + 1)
        l1 = -(4.0 / h[d] ** 2) * np.sin(j * math.pi * h[d] / 2) ** 2
        sh = [1] * len(shape)
        sh[len(shape) - 1 - d] = n
        lam = lam + l1.reshape(sh)
    return lam


def dst_apply(shape, h, fvals, v):
    V = v.reshape(shape[::-1])
    return F.dstn(fvals * F.dstn(V, type=1, norm="ortho"), type=1, norm="ortho").reshape(-1)


def dct_eigvals(shape, h):
    lam = 0.0
    for d, n in enumerate(shape):
        j = np.arange(n)
        l1 = -(4.0 / h[d] ** 2) * np.sin(j * math.pi / (2 * n)) ** 2
        sh = [1] * len(shape)
        sh[len(shape) - 1 - d] = n
        lam = lam + l1.reshape(sh)
    return lam


def dct_apply(shape, fvals, v):
    V = v.reshape(shape[::-1])
    return F.idctn(fvals * F.dctn(V, type=2, norm="ortho"), type=2, norm="ortho").reshape(-1)


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def augmented_phi1(A, tau, v):
    """phi_1(tau A) v as the top-right column of expm([[tau A, v], [0, 0]])."""
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = tau * A.toarray()
    M[:n, n] = v
    return sla.expm(M)[:n, n]


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_2d_dirichlet_128_dst_closed_form():
    """The small 2D workload: 128^2 interior, h = 1/129, tau = 1e-4, tol 1e-10."""
    N = 128
    h = 1.0 / (N + 1)
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    v = synth.uniform_vector(N * N, 0)
    y, st = I.phi_action(A, 1, 1e-4, v, 1e-10)
    want = dst_apply((N, N), (h, h), phi_scalar(1, 1e-4 * dst_eigvals((N, N), (h, h))), v)
    assert relerr(y, want) <= 1e-10
    assert st.converged and st.substeps == 1
    assert st.interval == (pytest.approx(-133128.0, rel=1e-14), pytest.approx(0.0, abs=1e-9))


@pytest.mark.parametrize("N,tau", [(40, 2e-2), (64, 1e-2), (33, 5e-2)])
def test_2d_dirichlet_substeps_dst(N, tau):
    h = 1.0 / (N + 1)
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    v = synth.uniform_vector(N * N, 7)
    y, st = I.phi_action(A, 1, tau, v, 1e-10)
    want = dst_apply((N, N), (h, h), phi_scalar(1, tau * dst_eigvals((N, N), (h, h))), v)
    assert st.substeps > 1
    assert relerr(y, want) <= 1e-10


@pytest.mark.parametrize("k", [0, 2])
def test_phi0_and_phi2_dst(k):
    N = 30
    h = 1.0 / (N + 1)
    tau = 5e-3
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    v = synth.uniform_vector(N * N, 3)
    y, st = I.phi_action(A, k, tau, v, 1e-11)
    want = dst_apply((N, N), (h, h), phi_scalar(k, tau * dst_eigvals((N, N), (h, h))), v)
    assert relerr(y, want) <= 1e-10


def test_single_eigenmode():
    """v = sin(j pi x) sin(k pi y) gives phi_1(tau lambda_jk) v exactly."""
    N = 50
    h = 1.0 / (N + 1)
    x = synth.interior_nodes(N)
    jj, kk = 3, 7
    v = (np.sin(kk * math.pi * x)[:, None] * np.sin(jj * math.pi * x)[None, :]).reshape(-1)
    lam = -(4 / h ** 2) * (math.sin(jj * math.pi * h / 2) ** 2 + math.sin(kk * math.pi * h / 2) ** 2)
    tau = 2e-3
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    y, _ = I.phi_action(A, 1, tau, v, 1e-12)
    assert relerr(y, math.expm1(tau * lam) / (tau * lam) * v) <= 1e-11


def test_3d_neumann_constant_dct_closed_form():
    n = (10, 12, 8)
    h = tuple(1.0 / s for s in n)
    tau = 2e-3
    A = O.stencil_matrix(n, h, "neumann0")
    v = synth.uniform_vector(int(np.prod(n)), 11)
    y, _ = I.phi_action(A, 1, tau, v, 1e-11)
    want = dct_apply(n, phi_scalar(1, tau * dct_eigvals(n, h)), v)
    assert relerr(y, want) <= 1e-10


def test_3d_dirichlet_dst_closed_form():
    n = (9, 7, 11)
    h = tuple(1.0 / (s + 1) for s in n)
    tau = 3e-3
    A = O.stencil_matrix(n, h, "dirichlet0")
    v = synth.uniform_vector(int(np.prod(n)), 12)
    y, _ = I.phi_action(A, 1, tau, v, 1e-11)
    want = dst_apply(n, h, phi_scalar(1, tau * dst_eigvals(n, h)), v)
    assert relerr(y, want) <= 1e-10


# ---------------------------------------------------------------------------
# brute force and an independent library algorithm
# ---------------------------------------------------------------------------

def test_variable_coefficient_neumann_brute_force():
    n = 8
    h = 1.0 / n
    coef = synth.sine_coefficient(n, 0.5).field()
    A = O.stencil_matrix((n, n, n), (h, h, h), "neumann0", coef=coef)
    v = synth.uniform_vector(n ** 3, 2)
    a, b = O.gershgorin_interval(A)
    tau = 60.0 / (b - a)
    y, st = I.phi_action(A, 1, tau, v, 1e-11)
    assert relerr(y, augmented_phi1(A, tau, v)) <= 1e-10
    # also through the eigendecomposition (A is symmetric)
    lam, Q = np.linalg.eigh(A.toarray())
    assert relerr(y, Q @ (phi_scalar(1, tau * lam) * (Q.T @ v))) <= 1e-10


def test_graph_laplacian_brute_force():
    g = synth.rgg_negative_laplacian(600, seed=9, mean_degree=20.0)
    A = O.csr_matrix(g.n, g.rowptr, g.colind, g.val)
    rho = synth.spectral_radius_symmetric(g)
    tau = 50.0 / rho
    v = synth.uniform_vector(g.n, 5)
    y, st = I.phi_action(A, 1, tau, v, 1e-11)
    assert relerr(y, augmented_phi1(A, tau, v)) <= 1e-10


def test_expm_multiply_variable_coefficient():
    """scipy's expm_multiply (truncated Taylor with scaling) on the sparse
    augmented matrix, a 20^3 variable-coefficient Neumann operator."""
    n = 20
    h = 1.0 / n
    coef = synth.sine_coefficient(n, 0.5).field()
    A = O.stencil_matrix((n, n, n), (h, h, h), "neumann0", coef=coef)
    v = synth.uniform_vector(n ** 3, 8)
    tau = 1e-3
    y, st = I.phi_action(A, 1, tau, v, 1e-12)
    N = A.shape[0]
    M = sp.bmat([[tau * A, sp.csr_matrix(v.reshape(-1, 1))],
                 [sp.csr_matrix((1, N)), sp.csr_matrix((1, 1))]], format="csr")
    e = np.zeros(N + 1)
    e[N] = 1.0
    want = expm_multiply(M, e)[:N]
    assert relerr(y, want) <= 1e-10


def test_scalar_operator():
    """A 1x1 operator lambda on a supplied interval: the whole machinery
    (Leja points, divided differences, Newton loop, stop test) must return
    expm1(tau lambda)/(tau lambda)."""
    a, b = -5000.0, 0.0
    for lam in (-5000.0, -3210.5, -1.0, 0.0):
        A = sp.csr_matrix(np.array([[lam]]))
        for tau in (1e-3, 2e-2):
            y, st = I.phi_action(A, 1, tau, np.array([1.0]), 1e-12, interval=(a, b))
            want = 1.0 if lam == 0 else math.expm1(tau * lam) / (tau * lam)
            assert y[0] == pytest.approx(want, rel=1e-10, abs=1e-14)


def test_zero_vector():
    A = O.stencil_matrix((6, 6), (0.1, 0.1), "dirichlet0")
    y, st = I.phi_action(A, 1, 1e-3, np.zeros(36), 1e-10)
    assert np.all(y == 0.0) and st.converged


def test_nonconvergence_doubles_substeps():
    N = 20
    h = 1.0 / (N + 1)
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    v = synth.uniform_vector(N * N, 1)
    tau = 60.0 / (8.0 / h ** 2)
    params = I.LejaParams(l_max=1000.0, m_max=20, max_retries=4)
    y, st = I.phi_action(A, 1, tau, v, 1e-10, params=params)
    assert st.retries >= 1 and st.converged
    want = dst_apply((N, N), (h, h), phi_scalar(1, tau * dst_eigvals((N, N), (h, h))), v)
    assert relerr(y, want) <= 1e-9


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def _neumann_var(n=9, amp=0.7):
    h = 1.0 / n
    coef = synth.sine_coefficient(n, amp).field()
    return O.stencil_matrix((n, n, n), (h, h, h), "neumann0", coef=coef)


def test_invariants_mass_symmetry_constants_positivity_linearity():
    A = _neumann_var()
    n = A.shape[0]
    a, b = O.gershgorin_interval(A)
    tau = 40.0 / (b - a)
    v = synth.uniform_vector(n, 21)
    w = synth.uniform_vector(n, 22)
    tol = 1e-12
    pv, _ = I.phi_action(A, 1, tau, v, tol)
    pw, _ = I.phi_action(A, 1, tau, w, tol)
    # mass: 1^T phi_1(tau A) v = 1^T v since 1^T A = 0
    assert abs(pv.sum() - v.sum()) <= 1e-10 * np.abs(v).sum()
    # symmetry
    assert abs(w @ pv - v @ pw) <= 1e-10 * np.linalg.norm(v) * np.linalg.norm(w)
    # constants are fixed points
    one, _ = I.phi_action(A, 1, tau, np.ones(n), tol)
    assert np.max(np.abs(one - 1.0)) <= 1e-10
    # positivity (A is Metzler)
    pos, _ = I.phi_action(A, 1, tau, np.abs(v), tol)
    assert pos.min() >= -1e-10 * np.abs(pos).max()
    # linearity
    pl, _ = I.phi_action(A, 1, tau, 2.0 * v - 3.0 * w, tol)
    assert relerr(pl, 2.0 * pv - 3.0 * pw) <= 1e-10


# ---------------------------------------------------------------------------
# exponential Euler
# ---------------------------------------------------------------------------

def test_expeuler_constant_forcing_is_exact():
    """For g == const b the exponential Euler step is exact:
    u1 = e^{tau A} u0 + tau phi_1(tau A) b (checked in the DST basis)."""
    N = 36
    h = 1.0 / (N + 1)
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    u0 = synth.uniform_vector(N * N, 4)
    bvec = np.full(N * N, 0.75)
    for tau in (1e-4, 3e-3):
        u1, st = I.expeuler_step(A, tau, u0, 1e-12, g=lambda u: bvec)
        lam = tau * dst_eigvals((N, N), (h, h))
        want = dst_apply((N, N), (h, h), np.exp(lam), u0) + tau * dst_apply(
            (N, N), (h, h), phi_scalar(1, lam), bvec)
        assert relerr(u1, want) <= 1e-10


def test_expeuler_cubic_brute_force_and_mass():
    A = _neumann_var(n=7, amp=0.5)
    n = A.shape[0]
    x = synth.gaussian_bump_3d(7, seed=3)
    a, b = O.gershgorin_interval(A)
    tau = 30.0 / (b - a)
    u1, st = I.expeuler_step(A, tau, x, 1e-12)
    g = x - x ** 3
    M = tau * A.toarray()
    want = sla.expm(M) @ x + tau * augmented_phi1(A, tau, g)
    assert relerr(u1, want) <= 1e-10
    # mass identity under Neumann: 1^T u1 = 1^T u0 + tau 1^T g(u0)
    assert abs(u1.sum() - (x.sum() + tau * g.sum())) <= 1e-11 * np.abs(x).sum()


def test_expeuler_substeps_match_single_step_form():
    """With several substeps the result still equals u + tau phi_1(tau A) F(u)."""
    N = 24
    h = 1.0 / (N + 1)
    A = O.stencil_matrix((N, N), (h, h), "dirichlet0")
    u0 = 0.5 * synth.uniform_vector(N * N, 6)
    tau = 300.0 / (8 / h ** 2)
    u1, st = I.expeuler_step(A, tau, u0, 1e-12)
    assert st.substeps >= 3
    Fu = A @ u0 + u0 - u0 ** 3
    want = u0 + tau * dst_apply((N, N), (h, h), phi_scalar(1, tau * dst_eigvals((N, N), (h, h))), Fu)
    assert relerr(u1, want) <= 1e-10


# ---------------------------------------------------------------------------
# the closed-form sine-mode phi_k of the oracle (used for large batched grids)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("shape,coef,tau", [((5, 4), 1.0, 3e-2), ((3, 4, 5), 0.7, 1e-2), ((7, 1), 2.0, 5e-2)])
def test_dirichlet_box_phi_matches_dense_brute_force(k, shape, coef, tau):
    """Against phi_k of the dense matrix: expm of tau A (k = 0), the augmented
    matrix for k = 1, and the (k+1)-block augmented matrix for k = 2."""
    h = tuple(1.0 / (s + 1.0) for s in shape)
    A = O.stencil_matrix(shape, h, "dirichlet0", coef=coef).toarray()
    n = A.shape[0]
    v = synth.uniform_vector(n, 4)
    got = O.dirichlet_box_phi(k, shape, h, tau, v, coef=coef)
    # phi_k(tau A) v = top-right block of expm([[tau A, v e_1^T, 0], [0, J]]) with a
    # Jordan shift block J of size k: the last column of the first block row
    M = np.zeros((n + k, n + k))
    M[:n, :n] = tau * A
    if k >= 1:
        M[:n, n] = v
        for q in range(k - 1):
            M[n + q, n + q + 1] = 1.0
        want = sla.expm(M)[:n, n + k - 1]
    else:
        want = sla.expm(M) @ v
    assert relerr(got, want) <= 1e-12


def test_phi_values_series_and_recurrence_agree_with_mpmath_values():
    from oracle import leja as L
    z = np.array([-40.0, -3.0, -1.0, -0.999, -0.3, -1e-7, 0.0, 1e-9, 0.5, 0.9999, 1.0, 2.5])
    for k in (1, 2, 3):
        got = O.phi_values(k, z)
        want = np.array([L.phi(k, float(t)) for t in z])
        assert np.allclose(got, want, rtol=2e-14, atol=0), k
