"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws and lays out input data: random vectors, initial
conditions, coefficient samples, sparse-matrix structure and the instance
table of the batched workload.  It contains none of the arithmetic of the
exponential-integrator method (no interval, no Leja points, no divided
differences, no stencil application), so both the CPU oracle and the HIP
path can consume its output without sharing any of the method's code.

Layout conventions (all arrays are C-contiguous numpy arrays):

* 2D grid vectors have shape ``(ny, nx)`` flattened with x fastest
  (flat index ``i + nx*j``).
* 3D grid vectors have shape ``(nz, ny, nx)`` flattened with x fastest
  (flat index ``i + nx*(j + ny*k)``).

Every generator takes an integer ``seed`` and builds its stream with
``numpy.random.default_rng(numpy.random.SeedSequence(seed))``, so a given
seed always reproduces the same bytes on any host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


# ---------------------------------------------------------------------------
# Vectors and initial conditions
# ---------------------------------------------------------------------------

def uniform_vector(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """``n`` float64 values drawn uniformly from ``[lo, hi)``."""
    return _rng(seed).uniform(lo, hi, size=int(n)).astype(np.float64)


def cell_centres(n: int) -> np.ndarray:
    """Cell-centre coordinates ``(i + 1/2)/n``, ``i = 0..n-1``, of the unit interval."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def interior_nodes(n: int) -> np.ndarray:
    """Interior node coordinates ``i/(n+1)``, ``i = 1..n``, of the unit interval."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def gaussian_bump_3d(n: int, seed: int = 0, sigma: float = 0.1,
                     noise: float = 0.01) -> np.ndarray:
    """Initial condition on the ``n^3`` cell-centred grid of the unit cube.

    ``u0 = exp(-|x - c|^2 / (2 sigma^2)) + noise * N(0, 1)`` with the centre
    ``c = (1/2, 1/2, 1/2)``; one standard-normal draw per cell, in flat order.
    Returned flattened, x fastest.
    """
    x = cell_centres(n) - 0.5
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2
    bump = np.exp(-r2 / (2.0 * sigma * sigma))
    eps = _rng(seed).standard_normal(size=n * n * n)
    return (bump.reshape(-1) + noise * eps).astype(np.float64)


# ---------------------------------------------------------------------------
# Coefficient samples
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class SeparableCoefficient:
    """Samples of ``a(x,y,z) = c0 + c1 * X(x) * Y(y) * Z(z)`` at grid points.

    ``tx``, ``ty``, ``tz`` hold ``X``, ``Y``, ``Z`` sampled at the grid
    coordinates of each axis; ``field()`` expands them to a full grid array
    (flattened, x fastest) as ``c0 + c1 * (tx[i] * ty[j] * tz[k])``.
    """

    c0: float
    c1: float
    tx: np.ndarray
    ty: np.ndarray
    tz: np.ndarray

    def field(self) -> np.ndarray:
        prod = (self.tz[:, None, None] * self.ty[None, :, None]) * self.tx[None, None, :]
        return (self.c0 + self.c1 * prod).reshape(-1).astype(np.float64)


def sine_coefficient(n: int, amp: float) -> SeparableCoefficient:
    """``a = 1 + amp * sin(2 pi x) sin(2 pi y) sin(2 pi z)`` at the cell centres
    of the ``n^3`` grid of the unit cube."""
    s = np.sin(2.0 * math.pi * cell_centres(n))
    return SeparableCoefficient(1.0, float(amp), s.copy(), s.copy(), s.copy())


def diffusivity_amplitudes(count: int, seed: int = 0, lo: float = 0.1,
                           hi: float = 0.9) -> np.ndarray:
    """Per-trajectory diffusivity amplitudes drawn uniformly from ``[lo, hi)``."""
    return _rng(seed).uniform(lo, hi, size=int(count))


def combustion_initial(n_points: int, seed: int = 0, noise: float = 0.0) -> np.ndarray:
    """Initial state of the combustion model: ``u0 = 1`` at every grid point
    (the paper leaves it unstated), plus ``noise * U[-1, 1)`` per point when
    ``noise > 0`` (so that tests see a state that is not constant)."""
    u = np.ones(int(n_points), dtype=np.float64)
    if noise > 0:
        u += noise * uniform_vector(n_points, seed)
    return u


# ---------------------------------------------------------------------------
# Unstructured matrix: negative graph Laplacian of a random geometric graph
# ---------------------------------------------------------------------------

@dataclass
class CsrMatrix:
    """A square CSR matrix with int32 indices and float64 values."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray     # float64[nnz]
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _morton_keys(pts: np.ndarray, bits: int = 10) -> np.ndarray:
    q = np.minimum((pts * (1 << bits)).astype(np.uint64), (1 << bits) - 1)
    key = np.zeros(len(pts), dtype=np.uint64)
    for b in range(bits):
        for d in range(3):
            key |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return key


def rgg_negative_laplacian(n: int, seed: int = 0, mean_degree: float = 26.0,
                           morton: bool = True) -> CsrMatrix:
    """Negative graph Laplacian ``W - D`` of a seeded random geometric graph.

    ``n`` points are drawn uniformly in the unit cube (not periodic).  Two
    distinct points are joined when their Euclidean distance is below
    ``r = (3 * mean_degree / (4 pi n))^(1/3)``, which gives about
    ``mean_degree`` neighbours per interior point (fewer near the faces), so
    about ``mean_degree + 1`` stored entries per row.  ``W`` has unit weights,
    ``D = diag(row sums of W)``.  With ``morton=True`` the points are renumbered
    in Morton (Z-curve) order first, which keeps neighbours close in index.
    Columns are sorted within each row; the diagonal entry is stored even for
    isolated points.
    """
    from scipy.spatial import cKDTree
    import scipy.sparse as sp

    pts = _rng(seed).uniform(0.0, 1.0, size=(int(n), 3))
    if morton:
        pts = pts[np.argsort(_morton_keys(pts), kind="stable")]
    r = (3.0 * mean_degree / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    deg = np.bincount(i, minlength=n).astype(np.float64)
    rows = np.concatenate([i, np.arange(n)])
    cols = np.concatenate([j, np.arange(n)])
    vals = np.concatenate([np.ones(len(i)), -deg])
    m = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    meta = {"radius": r, "mean_degree_target": mean_degree,
            "nnz_per_row": m.nnz / n, "max_degree": float(deg.max()), "morton": morton}
    return CsrMatrix(int(n), m.indptr.astype(np.int32), m.indices.astype(np.int32),
                     m.data.astype(np.float64), meta)


def spectral_radius_symmetric(csr: CsrMatrix, tol: float = 1e-6) -> float:
    """Largest |eigenvalue| of a symmetric CSR matrix by Lanczos (ARPACK).

    Used only to pick a time step with a prescribed stiffness ``tau * rho``.
    """
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh

    m = sp.csr_matrix((csr.val, csr.colind, csr.rowptr), shape=(csr.n, csr.n))
    # the all-ones vector is in the null space of a graph Laplacian, so the
    # Lanczos start vector is a fixed-seed random one
    v0 = _rng(12345).uniform(-1.0, 1.0, size=csr.n)
    lam = eigsh(m, k=1, which="LM", tol=tol, return_eigenvectors=False, v0=v0)
    return float(abs(lam[0]))


# ---------------------------------------------------------------------------
# Batched workload: many uneven 2D problems
# ---------------------------------------------------------------------------

@dataclass
class BatchInstance:
    n: int          # interior points per side (grid is n x n)
    tau: float      # time step
    seed: int       # seed of this instance's input vector

    def vector(self) -> np.ndarray:
        return uniform_vector(self.n * self.n, self.seed)


# ---------------------------------------------------------------------------
# Complex Hermitian matrix: a spin system in a spin bath
# ---------------------------------------------------------------------------

def spin_bath_hamiltonian(n_spins: int, seed: int = 0, n_central: int = 2,
                          bath_bonds: int = 40, anisotropy: float = 0.5,
                          field: float = 0.3) -> CsrMatrix:
    """Hermitian H (complex128 values) of ``n_spins`` spins 1/2 in the S^z
    basis (basis state index = bit pattern, bit i = spin i up), stored as CSR
    with int32 indices and sorted columns.  The paper's spin-bath matrix is
    not given; this one has its shape and sparsity: ``n_central`` central
    spins coupled to every bath spin, plus ``bath_bonds`` random bath-bath
    bonds, each bond (i, j) contributing

        J/2 (e^{i theta} S+_i S-_j + e^{-i theta} S-_i S+_j) + J Delta Sz_i Sz_j

    with J ~ U[-1, 1], theta ~ U[0, 2 pi), Delta = ``anisotropy``, plus a
    field h_i Sz_i, h_i ~ U[-field, field].  A flip term connects two states
    whose bits i and j differ, so a row holds about 1 + bonds/2 entries (21
    spins with 38 + 40 bonds: about 40 per row, as in the paper's 2^21
    matrix with 83.9 million entries).  The values are drawn from the seed;
    the numbers of the matrix are the Hamiltonian's definition, nothing of the
    integration method."""
    rng = _rng(seed)
    n = 1 << int(n_spins)
    bonds = [(c, b) for c in range(n_central) for b in range(n_central, n_spins)]
    bath = list(range(n_central, n_spins))
    seen = set(bonds)
    while len(bonds) < n_central * (n_spins - n_central) + bath_bonds and len(bath) >= 2:
        i, j = sorted(rng.choice(bath, size=2, replace=False).tolist())
        if (i, j) not in seen:
            seen.add((i, j))
            bonds.append((i, j))
    J = rng.uniform(-1.0, 1.0, size=len(bonds))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=len(bonds))
    h = rng.uniform(-field, field, size=n_spins)
    states = np.arange(n, dtype=np.int64)
    spin = lambda i: ((states >> i) & 1).astype(np.float64) - 0.5      # S^z eigenvalue
    diag = np.zeros(n)
    for i in range(n_spins):
        diag += h[i] * spin(i)
    nb = len(bonds)
    cols = np.full((n, nb + 1), -1, dtype=np.int64)
    vals = np.zeros((n, nb + 1), dtype=np.complex128)
    for q, ((i, j), Jq, tq) in enumerate(zip(bonds, J, theta)):
        si, sj = spin(i), spin(j)
        diag += Jq * anisotropy * si * sj
        # <new| S+_i S-_j |old> = 1 when spin i is down and spin j up in |old>
        mask = (1 << i) | (1 << j)
        # row r = new state: H[new, old] = J/2 e^{i theta} for the raising of i
        raised = (si > 0) & (sj < 0)          # new states reached by S+_i S-_j
        cols[raised, q] = states[raised] ^ mask
        vals[raised, q] = 0.5 * Jq * np.exp(1j * tq)
        lowered = (si < 0) & (sj > 0)         # new states reached by S-_i S+_j
        cols[lowered, q] = states[lowered] ^ mask
        vals[lowered, q] = 0.5 * Jq * np.exp(-1j * tq)
    cols[:, nb] = states
    vals[:, nb] = diag
    order = np.argsort(np.where(cols < 0, n, cols), axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    keep = cols >= 0
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CsrMatrix(n, rowptr.astype(np.int32), cols[keep].astype(np.int32),
                     vals[keep], {"spins": n_spins, "bonds": bonds, "J": J, "theta": theta,
                                  "h": h, "anisotropy": anisotropy, "kind": "spin bath"})


def complex_uniform_vector(n: int, seed: int = 0) -> np.ndarray:
    """complex128 values with real and imaginary parts uniform in [-1, 1)."""
    r = _rng(seed).uniform(-1.0, 1.0, size=(int(n), 2))
    return (r[:, 0] + 1j * r[:, 1]).astype(np.complex128)


def batched_instances(count: int = 256, seed: int = 0, nmin: int = 64,
                      nmax: int = 1024, tau_lo: float = 1e-5,
                      tau_hi: float = 1e-3) -> list[BatchInstance]:
    """Instance table of independent square 2D problems.

    Side lengths are log-uniform between ``nmin`` and ``nmax``
    (``n = round(nmin * (nmax/nmin)^U)``, ``U ~ U[0,1)``), time steps uniform
    in ``[tau_lo, tau_hi)``; instance ``i`` draws its vector from the
    sub-seed ``seed * 100003 + 1 + i``.
    """
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, size=count)
    taus = rng.uniform(tau_lo, tau_hi, size=count)
    ns = np.rint(nmin * (nmax / nmin) ** u).astype(int)
    return [BatchInstance(int(ns[i]), float(taus[i]), seed * 100003 + 1 + i)
            for i in range(count)]
