"""Operators A, the product (alpha A + beta I) x, and the Gershgorin interval.

Test infrastructure only (see the package docstring).

Stencil operators (Sec. III-A, the seven-point formula; Sec. III-B for a
position-dependent coefficient).  The paper writes the constant-coefficient
Laplacian; with a coefficient ``a`` this oracle uses the conservative form
div(a grad u) with face coefficients equal to the mean of the two adjacent
grid values::

    (A u)_c = sum over axes d, directions s = +-1 of
              a_{c, c+s e_d} * (u_{c+s e_d} - u_c) / h_d^2

with ``a_{c,c'} = (a_c + a_{c'}) / 2``.  Boundary handling is folded into A
(Sec. II-C, "the boundary conditions are incorporated into the matrix A"):

* ``dirichlet0``   - homogeneous Dirichlet: a neighbour outside the array has
  value 0; its face coefficient is taken as ``a_c`` (the cell's own value).
* ``neumann0``     - homogeneous Neumann (zero flux): faces on the boundary
  carry no flux, so out-of-array neighbours simply drop out.
* ``interior_only``- Sec. III-A's first option: only points whose whole
  stencil lies inside the array are updated; rows of the outermost layer of
  the array are zero.

With a = 1 and dirichlet0, ``h^2 (A u)`` is exactly the seven-point formula of
Sec. III-A (five-point in 2D).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

BCS = ("dirichlet0", "neumann0", "interior_only")


def stencil_matrix(shape, h, bc: str, coef=None) -> sp.csr_matrix:
    """Assemble the stencil operator as a CSR matrix.

    ``shape`` is ``(nx,)``, ``(nx, ny)`` or ``(nx, ny, nz)`` (x fastest in the
    flat index), ``h`` the grid spacing per axis (same length as ``shape``),
    ``coef`` either None (a = 1), a scalar, or a flat float64 array with one
    value per grid point.
    """
    if bc not in BCS:
        raise ValueError(f"unknown boundary condition {bc!r}")
    shape = tuple(int(s) for s in shape)
    h = tuple(float(x) for x in h)
    dim = len(shape)
    n = int(np.prod(shape))
    # numpy axis order is reversed: index [k, j, i] with i = x fastest
    np_shape = shape[::-1]
    idx = np.arange(n).reshape(np_shape)
    if coef is None:
        a = np.ones(n)
    elif np.isscalar(coef):
        a = np.full(n, float(coef))
    else:
        a = np.asarray(coef, dtype=np.float64).reshape(-1)
        if a.size != n:
            raise ValueError("coefficient has the wrong size")
    a_grid = a.reshape(np_shape)

    if bc == "interior_only":
        inner = np.ones(np_shape, dtype=bool)
        for ax in range(dim):
            sl = [slice(None)] * dim
            sl[ax] = 0
            inner[tuple(sl)] = False
            sl[ax] = -1
            inner[tuple(sl)] = False

    rows, cols, vals = [], [], []
    diag = np.zeros(np_shape)
    for d in range(dim):            # physical axis d (0 = x)
        ax = dim - 1 - d            # numpy axis of physical axis d
        inv_h2 = 1.0 / (h[d] * h[d])
        for s in (-1, +1):
            # points c whose neighbour c + s e_d exists in the array
            src = [slice(None)] * dim
            dst = [slice(None)] * dim
            if s == +1:
                src[ax] = slice(0, np_shape[ax] - 1)
                dst[ax] = slice(1, np_shape[ax])
            else:
                src[ax] = slice(1, np_shape[ax])
                dst[ax] = slice(0, np_shape[ax] - 1)
            src, dst = tuple(src), tuple(dst)
            c_idx = idx[src]
            nb_idx = idx[dst]
            face = 0.5 * (a_grid[src] + a_grid[dst]) * inv_h2
            if bc == "interior_only":
                keep = inner[src]
                c_idx, nb_idx, face = c_idx[keep], nb_idx[keep], face[keep]
                np.subtract.at(diag, np.unravel_index(c_idx, np_shape), face)
            else:
                diag[src] -= face
            rows.append(c_idx.reshape(-1))
            cols.append(nb_idx.reshape(-1))
            vals.append(face.reshape(-1))
            if bc == "dirichlet0":
                # the face towards the missing neighbour (value 0)
                edge = [slice(None)] * dim
                edge[ax] = -1 if s == +1 else 0
                diag[tuple(edge)] -= a_grid[tuple(edge)] * inv_h2
    rows.append(idx.reshape(-1))
    cols.append(idx.reshape(-1))
    vals.append(diag.reshape(-1))
    m = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    m.sum_duplicates()
    m.sort_indices()
    return m


def csr_matrix(n, rowptr, colind, val) -> sp.csr_matrix:
    """Wrap CSR arrays (int32 indices, float64 values) as a scipy matrix."""
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(colind), np.asarray(rowptr)),
                         shape=(int(n), int(n)))


def apply_op(A, alpha: float, beta: float, x: np.ndarray) -> np.ndarray:
    """The product (alpha A + beta I) x of eq. (3)."""
    return alpha * (A @ x) + beta * x


def gershgorin_interval(A) -> tuple[float, float]:
    """Real Gershgorin bound [a, b] for the spectrum (and, for symmetric A,
    the field of values) of A: ``a = min_i (A_ii - R_i)``,
    ``b = max_i (A_ii + R_i)`` with ``R_i = sum_{j != i} |A_ij|``.

    Sec. II-C requires an a-priori bound of the field of values; this is the
    bound used throughout.
    """
    A = sp.csr_matrix(A)
    d = A.diagonal()
    absA = abs(A)
    r = np.asarray(absA.sum(axis=1)).reshape(-1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def apply_at(shape, h, bc: str, u: np.ndarray, points, coef=None) -> np.ndarray:
    """``(A u)`` at the flat indices ``points``, evaluated one point at a time
    from the definition in the module docstring, without assembling A (for
    grids too large to assemble).  ``coef`` as in ``stencil_matrix``."""
    if bc not in BCS:
        raise ValueError(f"unknown boundary condition {bc!r}")
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    n = int(np.prod(shape))
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    if coef is None:
        a = lambda idx: 1.0
    elif np.isscalar(coef):
        a = lambda idx: float(coef)
    else:
        arr = np.asarray(coef, dtype=np.float64).reshape(-1)
        if arr.size != n:
            raise ValueError("coefficient has the wrong size")
        a = lambda idx: float(arr[idx])
    strides = [int(np.prod(shape[:d])) for d in range(dim)]
    out = np.empty(len(points))
    for q, flat in enumerate(points):
        flat = int(flat)
        pos = [(flat // strides[d]) % shape[d] for d in range(dim)]
        if bc == "interior_only" and any(p == 0 or p == s - 1 for p, s in zip(pos, shape)):
            out[q] = 0.0
            continue
        ac = a(flat)
        total = 0.0
        for d in range(dim):
            for s in (-1, +1):
                p = pos[d] + s
                if 0 <= p < shape[d]:
                    nb = flat + s * strides[d]
                    total += 0.5 * (ac + a(nb)) * (u[nb] - u[flat]) / (h[d] * h[d])
                elif bc == "dirichlet0":
                    total += ac * (0.0 - u[flat]) / (h[d] * h[d])
        out[q] = total
    return out


def phi_values(k: int, z) -> np.ndarray:
    """phi_k(z) elementwise in float64 (phi_0 = exp, phi_{j+1}(z) =
    (phi_j(z) - 1/j!) / z, phi_j(0) = 1/j!).  Near zero (|z| < 1) the Taylor
    series sum_i z^i / (i + k)! to 30 terms avoids the cancellation of the
    recurrence; elsewhere phi_1 = expm1(z)/z starts the recurrence."""
    import math
    z = np.asarray(z, dtype=np.float64)
    if k == 0:
        return np.exp(z)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    ser = np.zeros_like(zs)
    term = np.full_like(zs, 1.0 / math.factorial(k))
    for i in range(30):
        ser += term
        term = term * zs / (i + k + 1)
    out[small] = ser
    zb = z[~small]
    val = np.expm1(zb) / zb
    for j in range(1, k):
        val = (val - 1.0 / math.factorial(j)) / zb
    out[~small] = val
    return out


def dirichlet_box_phi(k: int, shape, h, tau: float, v: np.ndarray, coef: float = 1.0) -> np.ndarray:
    """Closed form of phi_k(tau A) v for A = coef times the constant-coefficient
    Laplacian (five- or seven-point formula, Sec. III-A) with homogeneous
    Dirichlet boundaries, ``h_d = 1/(n_d + 1)`` on every axis.

    The sine modes diagonalise A: the orthonormal DST-I along each axis maps
    v to mode coefficients, mode (j_1, j_2, ...) has the eigenvalue
    ``-coef * sum_d (4/h_d^2) sin^2(j_d pi / (2 (n_d + 1)))``, and phi_k of
    tau times it scales the coefficient.  Exact up to rounding; no Leja
    interpolation involved, so it checks the interpolation's result
    independently of its algorithm.  ``shape`` is (n_x, n_y[, n_z]) with x
    fastest in ``v``."""
    import scipy.fft as F
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    lam = 0.0
    for d in range(dim):
        j = np.arange(1, shape[d] + 1)
        l1 = -coef * (4.0 / (h[d] * h[d])) * np.sin(j * np.pi / (2.0 * (shape[d] + 1))) ** 2
        sh = [1] * dim
        sh[dim - 1 - d] = shape[d]
        lam = lam + l1.reshape(sh)
    V = np.asarray(v, dtype=np.float64).reshape(shape[::-1])
    modes = F.dstn(V, type=1, norm="ortho")
    return F.dstn(phi_values(k, tau * lam) * modes, type=1, norm="ortho").reshape(-1)
