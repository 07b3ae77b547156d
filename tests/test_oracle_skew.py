"""Pins of the oracle's complex (K = C) path: phi_k(-i tau H) v for Hermitian H.

Dense matrix exponentials, the eigendecomposition, a two-level closed form,
the sine-mode closed form for a real symmetric H, unitarity, and the
interpolation property of the complex divided differences.  Also the
spin-bath generator against a Kronecker-product construction.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from oracle import integrators as I
from oracle import leja as L
from oracle import operators as O


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_hermitian(n, seed, density=0.15):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M = np.where(rng.uniform(size=(n, n)) < density, M, 0.0)
    M = (M + M.conj().T) / 2
    return M


@pytest.mark.parametrize("length", [8.0, 90.0, 260.0])
def test_skew_exp_dense_expm(length):
    M = random_hermitian(70, 1)
    H = sp.csr_matrix(M)
    a, b = O.gershgorin_interval(H)
    tau = length / (b - a)
    v = synth.complex_uniform_vector(70, 2)
    y, st = I.skew_phi_action(H, 0, tau, v, 1e-12)
    want = sla.expm(-1j * tau * M) @ v
    assert st.converged and st.substeps == max(1, math.ceil(length / 100))
    assert relerr(y, want) <= 1e-10
    # e^{-i tau H} is unitary
    assert abs(np.linalg.norm(y) - np.linalg.norm(v)) <= 1e-10 * np.linalg.norm(v)


@pytest.mark.parametrize("length", [8.0, 150.0])
def test_skew_phi1_augmented_expm(length):
    M = random_hermitian(50, 3)
    H = sp.csr_matrix(M)
    a, b = O.gershgorin_interval(H)
    tau = length / (b - a)
    v = synth.complex_uniform_vector(50, 4)
    y, st = I.skew_phi_action(H, 1, tau, v, 1e-12)
    Aug = np.zeros((51, 51), dtype=np.complex128)
    Aug[:50, :50] = -1j * tau * M
    Aug[:50, 50] = v
    want = sla.expm(Aug)[:50, 50]
    assert relerr(y, want) <= 1e-10


def test_skew_eigh_and_two_level():
    M = random_hermitian(40, 5)
    lam, Q = np.linalg.eigh(M)
    v = synth.complex_uniform_vector(40, 6)
    a, b = O.gershgorin_interval(M)
    tau = 30.0 / (b - a)
    y, _ = I.skew_phi_action(sp.csr_matrix(M), 0, tau, v, 1e-12)
    assert relerr(y, Q @ (np.exp(-1j * tau * lam) * (Q.conj().T @ v))) <= 1e-10
    # two levels: e^{-i t H} = cos(w t) I - i sin(w t) H / w, w = sqrt(eps^2 + Omega^2)
    eps, Om = 0.3, 1.7
    H2 = np.array([[eps, Om], [Om, -eps]], dtype=np.complex128)
    w = math.hypot(eps, Om)
    psi = np.array([1.0, 0.0], dtype=np.complex128)
    for t in (0.1, 2.0, 7.5):
        y, _ = I.skew_phi_action(sp.csr_matrix(H2), 0, t, psi, 1e-13)
        want = math.cos(w * t) * psi - 1j * math.sin(w * t) * (H2 @ psi) / w
        assert np.max(np.abs(y - want)) <= 1e-11


def test_skew_real_symmetric_sine_modes():
    """H = the 2D Dirichlet Laplacian (real symmetric): e^{-i tau H} v by the
    sine transform with e^{-i tau lambda}."""
    import scipy.fft as F
    shape = (17, 13)
    h = tuple(1.0 / (s + 1) for s in shape)
    A = O.stencil_matrix(shape, h, "dirichlet0")
    a, b = O.gershgorin_interval(A)
    tau = 60.0 / (b - a)
    v = synth.complex_uniform_vector(A.shape[0], 7)
    y, _ = I.skew_phi_action(A, 0, tau, v, 1e-12)
    lam = 0.0
    for d in range(2):
        j = np.arange(1, shape[d] + 1)
        l1 = -(4.0 / h[d] ** 2) * np.sin(j * np.pi / (2.0 * (shape[d] + 1))) ** 2
        sh = [1, 1]
        sh[1 - d] = shape[d]
        lam = lam + l1.reshape(sh)
    V = v.reshape(shape[::-1])
    want = F.dstn(np.exp(-1j * tau * lam) * F.dstn(V, type=1, norm="ortho"), type=1, norm="ortho")
    assert relerr(y, want.reshape(-1)) <= 1e-10


@pytest.mark.parametrize("k", [0, 1])
def test_skew_divided_differences_interpolate(k):
    import mpmath
    xi = L.leja_points(40)
    delta, c, gamma = 0.7, -3.0, 5.0
    d = L.divided_differences_skew(k, delta, c, gamma, xi)
    for i in (0, 5, 17, 39):
        val = sum(d[j] * np.prod(xi[i] - xi[:j]) for j in range(40))
        with mpmath.workdps(40):
            want = complex(L.phi_mpc(k, mpmath.mpc(0, -1) * delta * (c + gamma * xi[i])))
        assert abs(val - want) <= 1e-12 * max(1.0, abs(want))


def test_spin_bath_generator_matches_kronecker_construction():
    n_spins = 6
    g = synth.spin_bath_hamiltonian(n_spins, seed=3, bath_bonds=4)
    H = sp.csr_matrix((g.val, g.colind, g.rowptr), shape=(g.n, g.n)).toarray()
    # single-spin operators in the basis (down, up) = (0, 1)
    Sz = np.diag([-0.5, 0.5]).astype(np.complex128)
    Sp = np.array([[0, 0], [1, 0]], dtype=np.complex128)
    Sm = Sp.T.copy()
    I2 = np.eye(2, dtype=np.complex128)

    def on(ops):
        # basis index = sum_i bit_i 2^i: spin 0 is the last Kronecker factor
        out = np.ones((1, 1), dtype=np.complex128)
        for i in range(n_spins - 1, -1, -1):
            out = np.kron(out, ops.get(i, I2))
        return out

    want = np.zeros_like(H)
    for (i, j), J, th in zip(g.meta["bonds"], g.meta["J"], g.meta["theta"]):
        want += 0.5 * J * (np.exp(1j * th) * on({i: Sp, j: Sm}) + np.exp(-1j * th) * on({i: Sm, j: Sp}))
        want += J * g.meta["anisotropy"] * on({i: Sz, j: Sz})
    for i, hi in enumerate(g.meta["h"]):
        want += hi * on({i: Sz})
    assert np.max(np.abs(H - want)) <= 1e-14
    assert np.all(np.diff(g.rowptr) >= 1)
    for r in range(g.n):
        c = g.colind[g.rowptr[r]:g.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)
