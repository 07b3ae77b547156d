"""Pins of the oracle's operator assembly, eq. (3) product and Gershgorin bound.

Each test ties ``oracle.operators`` to something other than itself: a
Kronecker-sum construction from 1D second differences, the continuous
operator div(a grad u) (second-order consistency), the energy identity of a
flux-form operator, the seven-point formula of Sec. III-A written per point,
dense eigenvalues, and brute-force distances for the graph.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import operators as O


def second_difference_1d(n, h, bc):
    """Textbook 1D second-difference matrix tridiag(1, -2, 1)/h^2 with
    Dirichlet (u = 0 beyond the ends) or zero-flux Neumann ends."""
    main = -2.0 * np.ones(n)
    if bc == "neumann0":
        main[0] = main[-1] = -1.0
    off = np.ones(n - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)


@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0"])
@pytest.mark.parametrize("shape", [(7,), (5, 9), (4, 6, 3)])
def test_constant_coefficient_is_kronecker_sum(shape, bc):
    h = [1.0 / (s + 1) for s in shape]
    A = O.stencil_matrix(shape, h, bc)
    # x fastest: flat index i + nx*j (+ nx*ny*k); Kronecker order is (z, y, x)
    K = None
    for d, (n, hd) in enumerate(zip(shape, h)):
        T = second_difference_1d(n, hd, bc)
        left = sp.identity(int(np.prod(shape[d + 1:]))) if d + 1 < len(shape) else sp.identity(1)
        right = sp.identity(int(np.prod(shape[:d]))) if d > 0 else sp.identity(1)
        term = sp.kron(sp.kron(left, T), right)
        K = term if K is None else K + term
    assert abs(A - K).max() < 1e-9 * abs(K).max()


def test_scalar_coefficient_scales_operator():
    shape, h = (6, 5, 4), (0.1, 0.2, 0.25)
    A1 = O.stencil_matrix(shape, h, "neumann0")
    A3 = O.stencil_matrix(shape, h, "neumann0", coef=3.0)
    assert abs(A3 - 3.0 * A1).max() < 1e-12 * abs(A3).max()


def test_seven_point_formula_interior_only():
    """Sec. III-A: (dx)^2 (Au) = -6u + the six neighbours, on the points whose
    stencil lies inside the array; rows of the outer layer are zero."""
    n = (6, 7, 5)
    dx = 0.1
    A = O.stencil_matrix(n, (dx, dx, dx), "interior_only")
    rng = np.random.default_rng(1)
    u = rng.standard_normal(int(np.prod(n)))
    got = (A @ u).reshape(n[::-1])
    U = u.reshape(n[::-1])
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                if 0 < i < n[0] - 1 and 0 < j < n[1] - 1 and 0 < k < n[2] - 1:
                    want = (-6 * U[k, j, i] + U[k, j, i + 1] + U[k, j, i - 1] + U[k, j + 1, i]
                            + U[k, j - 1, i] + U[k + 1, j, i] + U[k - 1, j, i]) / dx ** 2
                else:
                    want = 0.0
                assert abs(got[k, j, i] - want) <= 1e-9 * (1 + abs(want))


def test_variable_coefficient_neumann_second_order():
    """Cell-centred flux form approximates div(a grad u) to O(h^2) in the
    interior, for a = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z) and
    u = cos(pi x) cos(pi y) cos(pi z) (zero normal derivative on the faces)."""
    errs = []
    for n in (12, 24):
        h = 1.0 / n
        coef = synth.sine_coefficient(n, 0.5)
        A = O.stencil_matrix((n, n, n), (h, h, h), "neumann0", coef=coef.field())
        x = synth.cell_centres(n)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        pi = math.pi
        u = np.cos(pi * X) * np.cos(pi * Y) * np.cos(pi * Z)
        s2 = lambda t: np.sin(2 * pi * t)
        c2 = lambda t: np.cos(2 * pi * t)
        a = 1 + 0.5 * s2(X) * s2(Y) * s2(Z)
        ax = 0.5 * 2 * pi * c2(X) * s2(Y) * s2(Z)
        ay = 0.5 * 2 * pi * s2(X) * c2(Y) * s2(Z)
        az = 0.5 * 2 * pi * s2(X) * s2(Y) * c2(Z)
        ux = -pi * np.sin(pi * X) * np.cos(pi * Y) * np.cos(pi * Z)
        uy = -pi * np.cos(pi * X) * np.sin(pi * Y) * np.cos(pi * Z)
        uz = -pi * np.cos(pi * X) * np.cos(pi * Y) * np.sin(pi * Z)
        lap = -3 * pi * pi * u
        exact = a * lap + ax * ux + ay * uy + az * uz
        got = (A @ u.reshape(-1)).reshape(u.shape)
        inner = (slice(2, -2),) * 3
        errs.append(np.max(np.abs(got[inner] - exact[inner])))
    assert errs[1] < errs[0] / 3.2, errs


def test_flux_form_energy_identity_and_symmetry():
    """-u^T A u = sum over interior faces of a_face (u_c - u_c')^2 / h_d^2
    for the Neumann operator; A is symmetric with zero row sums."""
    n = (5, 4, 6)
    h = (0.2, 0.25, 0.5)
    rng = np.random.default_rng(3)
    a = 1.0 + rng.uniform(0, 1, size=int(np.prod(n)))
    A = O.stencil_matrix(n, h, "neumann0", coef=a)
    assert abs(A - A.T).max() == 0.0
    assert np.max(np.abs(np.asarray(A.sum(axis=1)))) < 1e-12 * abs(A).max()
    u = rng.standard_normal(int(np.prod(n)))
    U = u.reshape(n[::-1])
    Ag = a.reshape(n[::-1])
    energy = 0.0
    for d in range(3):
        ax = 2 - d
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        face = 0.5 * (Ag[tuple(sl_lo)] + Ag[tuple(sl_hi)])
        energy += np.sum(face * (U[tuple(sl_lo)] - U[tuple(sl_hi)]) ** 2) / h[d] ** 2
    assert abs(-u @ (A @ u) - energy) <= 1e-12 * energy


def test_dirichlet_variable_coefficient_boundary_faces():
    """Homogeneous Dirichlet with a coefficient: the face towards the missing
    neighbour (value 0) carries the cell's own coefficient, so A + (that
    diagonal) is the Neumann operator."""
    n = (4, 5)
    h = (0.3, 0.2)
    a = np.linspace(1.0, 2.0, 20)
    AD = O.stencil_matrix(n, h, "dirichlet0", coef=a)
    AN = O.stencil_matrix(n, h, "neumann0", coef=a)
    Ag = a.reshape(n[::-1])
    extra = np.zeros(n[::-1])
    extra[:, 0] += Ag[:, 0] / h[0] ** 2
    extra[:, -1] += Ag[:, -1] / h[0] ** 2
    extra[0, :] += Ag[0, :] / h[1] ** 2
    extra[-1, :] += Ag[-1, :] / h[1] ** 2
    diff = (AN - AD).toarray()
    assert np.allclose(diff, np.diag(extra.reshape(-1)), rtol=0, atol=1e-12)


def test_apply_op_is_eq3():
    A = O.stencil_matrix((5, 6), (0.1, 0.1), "dirichlet0")
    x = np.arange(30.0)
    y = O.apply_op(A, 2.5, -0.75, x)
    assert np.allclose(y, 2.5 * (A.toarray() @ x) - 0.75 * x, rtol=1e-14, atol=1e-10)


@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
def test_gershgorin_contains_spectrum(bc):
    rng = np.random.default_rng(5)
    n = (6, 5, 4)
    a = 1 + 0.9 * rng.uniform(-1, 1, size=120)
    A = O.stencil_matrix(n, (0.1, 0.2, 0.3), bc, coef=a)
    lo, hi = O.gershgorin_interval(A)
    ev = np.linalg.eigvals(A.toarray()).real
    assert ev.min() >= lo - 1e-9 * abs(lo)
    assert ev.max() <= hi + 1e-9 * abs(lo)
    assert hi <= 1e-9 * abs(lo)   # every A here is diagonally dominant with negative diagonal


def test_gershgorin_2d_dirichlet_closed_form():
    N = 128
    h = 1.0 / (N + 1)
    lo, hi = O.gershgorin_interval(O.stencil_matrix((N, N), (h, h), "dirichlet0"))
    assert lo == pytest.approx(-8.0 / h ** 2, rel=1e-14)
    assert lo == pytest.approx(-133128.0, rel=1e-14)
    assert abs(hi) <= 1e-9


def test_rgg_laplacian_brute_force():
    n = 300
    g = synth.rgg_negative_laplacian(n, seed=4, mean_degree=12.0, morton=True)
    A = O.csr_matrix(g.n, g.rowptr, g.colind, g.val).toarray()
    assert np.array_equal(A, A.T)
    assert np.all(A.sum(axis=1) == 0.0)
    # recover the points in the stored (Morton) order
    pts = np.random.default_rng(np.random.SeedSequence(4)).uniform(0, 1, size=(n, 3))
    pts = pts[np.argsort(synth._morton_keys(pts), kind="stable")]
    dist = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    adj = (dist < g.meta["radius"]) & ~np.eye(n, dtype=bool)
    assert np.array_equal(A - np.diag(np.diag(A)), adj.astype(float))
    assert np.array_equal(np.diag(A), -adj.sum(axis=1).astype(float))
    lo, hi = O.gershgorin_interval(O.csr_matrix(g.n, g.rowptr, g.colind, g.val))
    assert lo == -2 * adj.sum(axis=1).max() and hi == 0.0


@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
@pytest.mark.parametrize("shape", [(9, 7), (6, 5, 8)])
def test_apply_at_matches_assembled_matrix(bc, shape):
    rng = np.random.default_rng(17)
    n = int(np.prod(shape))
    h = tuple(0.1 * (d + 1) for d in range(len(shape)))
    coef = 1 + 0.5 * rng.uniform(size=n)
    u = rng.standard_normal(n)
    pts = rng.choice(n, size=40, replace=False)
    for c in (None, 2.0, coef):
        A = O.stencil_matrix(shape, h, bc, coef=c)
        want = (A @ u)[pts]
        got = O.apply_at(shape, h, bc, u, pts, coef=c)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
