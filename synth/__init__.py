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
