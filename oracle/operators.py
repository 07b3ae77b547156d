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

Grid positions (needed where data depend on position): index i along an
axis of spacing h sits at ``(i + 1) h`` under dirichlet0 (nodes strictly
inside the unit interval, boundary nodes at 0 and ``(n + 1) h``),
``(i + 1/2) h`` under neumann0 (cell centres) and ``i h`` under
interior_only (the array includes the boundary layer).

Two further operators of the paper:

* inhomogeneous Dirichlet data (Sec. III-A, the rows of Table I with
  boundary values f = z(1-z)xy and f = sin(pi z) exp(-xy)): the stencil reads
  f at a neighbour position on the boundary instead of 0, which makes the
  product affine, ``A_0 u + b_f``, with A_0 the dirichlet0 operator and b_f
  the boundary term (``dirichlet_boundary_term``);
* the position-dependent coefficient of Sec. III-B in the form the paper
  times (Table II), ``D(x, y, z) times the discrete Laplacian`` with
  ``D = 1/sqrt(1 + x^2 + y^2)`` (``dlap_matrix``).
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
    bound used throughout.  For a Hermitian A the same bound holds for its
    real spectrum.
    """
    A = sp.csr_matrix(A)
    d = A.diagonal()
    if np.iscomplexobj(d):
        # Hermitian A (K = C): the diagonal is real
        d = d.real
    absA = abs(A)
    r = np.asarray(absA.sum(axis=1)).reshape(-1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


def apply_at(shape, h, bc: str, u: np.ndarray, points, coef=None, bdata=None,
             dlap: bool = False) -> np.ndarray:
    """``(A u)`` at the flat indices ``points``, evaluated one point at a time
    from the definition in the module docstring, without assembling A (for
    grids too large to assemble).  ``coef`` as in ``stencil_matrix``.
    ``bdata``: Dirichlet data f (``boundary_values`` kind, dirichlet0, 3D):
    a missing neighbour reads f at its boundary position instead of 0, so
    the result is ``(A_0 u + b_f)``.  ``dlap``: the operator D times the
    Laplacian (``dlap_matrix``; coef must be None)."""
    if bdata is not None and (bc != "dirichlet0" or len(shape) != 3):
        raise ValueError("boundary data need dirichlet0 on a 3D grid")
    if dlap and coef is not None:
        raise ValueError("dlap takes no coefficient")
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
                    ghost = 0.0
                    if bdata is not None:
                        xyz = [(pos[e] + 1) * h[e] for e in range(3)]
                        xyz[d] = 0.0 if p < 0 else (shape[d] + 1) * h[d]
                        ghost = float(boundary_values(bdata, *xyz))
                    total += ac * (ghost - u[flat]) / (h[d] * h[d])
        if dlap:
            xy = [float(positions(shape[e], h[e], bc)[pos[e]]) for e in range(2)]
            total *= float(d_coefficient(xy[0], xy[1]))
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


def positions(n: int, h: float, bc: str) -> np.ndarray:
    """Coordinates of the n grid indices of one axis (module docstring)."""
    off = {"dirichlet0": 1.0, "neumann0": 0.5, "interior_only": 0.0}[bc]
    return (np.arange(n) + off) * h


def boundary_values(kind: str, x, y, z):
    """The boundary data of Sec. III-A: ``z1mz_xy`` is f = z(1-z)xy,
    ``sinpiz_expmxy`` is f = sin(pi z) exp(-x y)."""
    if kind == "z1mz_xy":
        return z * (1.0 - z) * x * y
    if kind == "sinpiz_expmxy":
        return np.sin(np.pi * z) * np.exp(-x * y)
    raise ValueError(f"unknown boundary data {kind!r}")


def dirichlet_boundary_term(shape, h, kind: str, coef=None) -> np.ndarray:
    """b_f of the affine product ``A_0 u + b_f`` for Dirichlet data f on the
    boundary of the unit cube (3D, node grid of dirichlet0).  For every grid
    point and every axis direction whose neighbour index falls outside the
    array, the neighbour is the boundary node at coordinate 0 or
    ``(n + 1) h`` on that axis, and the face term ``a_c f(neighbour) / h^2``
    (the cell's own coefficient on the boundary face, as for dirichlet0) is
    added at the point."""
    shape = tuple(int(s) for s in shape)
    if len(shape) != 3:
        raise ValueError("boundary data are defined on 3D grids")
    n = int(np.prod(shape))
    a = np.ones(n) if coef is None else (np.full(n, float(coef)) if np.isscalar(coef)
                                         else np.asarray(coef, np.float64).reshape(-1))
    a = a.reshape(shape[::-1])
    X = positions(shape[0], h[0], "dirichlet0")[None, None, :]
    Y = positions(shape[1], h[1], "dirichlet0")[None, :, None]
    Z = positions(shape[2], h[2], "dirichlet0")[:, None, None]
    out = np.zeros(shape[::-1])
    full = lambda v: np.broadcast_to(v, shape[::-1])
    for d, (lo, hi) in enumerate(((0.0, (shape[0] + 1) * h[0]), (0.0, (shape[1] + 1) * h[1]),
                                  (0.0, (shape[2] + 1) * h[2]))):
        ax = 2 - d
        for end, coord in ((0, lo), (-1, hi)):
            sl = [slice(None)] * 3
            sl[ax] = end
            sl = tuple(sl)
            xyz = [full(X), full(Y), full(Z)]
            xyz[d] = np.full(shape[::-1], coord)
            f = boundary_values(kind, xyz[0][sl], xyz[1][sl], xyz[2][sl])
            out[sl] += a[sl] * f / (h[d] * h[d])
    return out.reshape(-1)


def d_coefficient(x, y) -> np.ndarray:
    """D(x, y, z) = 1/sqrt(1 + x^2 + y^2) of Sec. III-B (Table II)."""
    return 1.0 / np.sqrt(1.0 + x * x + y * y)


def dlap_matrix(shape, h, bc: str) -> sp.csr_matrix:
    """D times the constant-coefficient stencil Laplacian with boundary
    handling ``bc`` (Sec. III-B, Table II): row c of the Laplacian scaled by
    D at c's position."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3):
        raise ValueError("2D or 3D grids")
    L = stencil_matrix(shape, h, bc)
    X = positions(shape[0], h[0], bc)
    Y = positions(shape[1], h[1], bc)
    if dim == 3:
        Dg = np.broadcast_to(d_coefficient(X[None, None, :], Y[None, :, None]), shape[::-1])
    else:
        Dg = d_coefficient(X[None, :], Y[:, None])
    return sp.csr_matrix(sp.diags(np.ascontiguousarray(Dg).reshape(-1)) @ L)
