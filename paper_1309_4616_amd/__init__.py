"""MI355X-native phi_k(tau A) v by real Leja-point Newton interpolation.

Python face of libexpi.so (Einkemmer & Ostermann, "Exponential Integrators on
Graphic Processing Units", HPCS 2013): operators (matrix-free stencils with
folded boundary conditions, CSR), the product (alpha A + beta I) x of
eq. (3), phi_k(tau A) v (Sec. II-C, III-C) and the exponential Euler step of
eq. (2).  Device memory and streams come from PyTorch; every computation runs
in the HIP library, and a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes

from . import autotune, selector
from ._binding import (BDATA, BDATA_MODES, COEF_CONST, COEF_DLAP, COEF_FIELD, COEF_SEPARABLE, F32, F64,
                       G_CUBIC, NONLIN, BCS, EXPORTS,
                       NOALLOC_SCRATCH_BYTES, BatchStat, ExpiError, LejaParams, Stats, check,
                       divided_differences, divided_differences_skew, leja_points, lib)

__all__ = ["StencilOp", "CsrOp", "CsrComplexOp", "skew_phi_action", "apply_op", "phi_action", "phi_action_noalloc", "noalloc_init",
           "expeuler_step", "exprk2_step", "nonlinearity", "leja_points",
           "divided_differences", "ExpiError", "LejaParams", "workspace", "F64", "F32",
           "autotune", "selector", "Batch"]


def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    torch = _torch()
    if dtype in ("f64", F64, torch.float64):
        return F64
    if dtype in ("f32", F32, torch.float32):
        return F32
    raise ValueError(f"dtype must be f64 or f32, got {dtype!r}")


def _stream_ptr(stream, device):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, device, n=None, name="array"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t, dtype=torch.float64)
    t = t.to(device=device, dtype=torch.float64).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t


class _Op:
    """Owns an expi_op handle and the device tensors it borrows."""

    def __init__(self):
        self._h = ctypes.c_void_p()
        self._keep = []
        self._ws = {}

    @property
    def handle(self):
        return self._h

    @property
    def size(self) -> int:
        return int(lib().expi_op_size(self._h))

    def workspace_bytes(self, dtype="f64") -> int:
        return int(lib().expi_workspace_bytes(self._h, _dtype_code(dtype)))

    def workspace(self, dtype="f64"):
        """A cached device workspace of the required size for this operator."""
        code = _dtype_code(dtype)
        ws = self._ws.get(code)
        if ws is None:
            ws = workspace(self.workspace_bytes(code), self.device)
            self._ws[code] = ws
        return ws

    def set_tiles(self, vec: int, waves: int, march: int) -> None:
        """Tile setting of the operator's sweeps (see expi_op_set_tiles)."""
        check(lib().expi_op_set_tiles(self._h, int(vec), int(waves), int(march)))

    def tiles(self) -> tuple:
        v, w, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().expi_op_get_tiles(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(m)))
        return v.value, w.value, m.value

    def set_pairs(self, use) -> None:
        """Pair sweeps where they apply (the default), or single products
        (see expi_op_set_pairs); on a 2D operator an int 4..64 (a multiple
        of 4) also sets the rows per tile of its pair sweep."""
        u = use if (isinstance(use, int) and not isinstance(use, bool) and use > 1) else (1 if use else 0)
        check(lib().expi_op_set_pairs(self._h, u))

    def pairs(self) -> bool:
        return bool(self.pair_setting())

    def pair_setting(self) -> int:
        """The stored pair setting: 0 off, 1 on, or the 2D pair sweep's rows
        per tile."""
        u = ctypes.c_int()
        check(lib().expi_op_get_pairs(self._h, ctypes.byref(u)))
        return int(u.value)

    def interval(self, stream=None):
        a, b = ctypes.c_double(), ctypes.c_double()
        ws = self.workspace("f64")
        check(lib().expi_op_interval(self._h, ctypes.byref(a), ctypes.byref(b),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream_ptr(stream, self.device)))
        return a.value, b.value

    def __del__(self):
        try:
            if self._h:
                lib().expi_op_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


class StencilOp(_Op):
    """Matrix-free 2D/3D stencil A = div(a grad .) with folded boundary handling.

    shape: (nx, ny) or (nx, ny, nz), x fastest; h: spacing per axis.
    bc: 'dirichlet0', 'neumann0' or 'interior_only'.
    coef: None (a = 1), a float (a = c0), a tuple ('separable', c0, c1, tx, ty[, tz])
    giving a = c0 + c1 tx[i] ty[j] tz[k], ('dlap', c0) for c0 D(x, y) times the
    Laplacian (D = 1/sqrt(1 + x^2 + y^2), Sec. III-B), or an array of the grid's size.
    """

    def __init__(self, shape, h, bc="dirichlet0", coef=None, device="cuda:0"):
        super().__init__()
        torch = _torch()
        self.device = torch.device(device)
        self.shape = tuple(int(s) for s in shape)
        self.h = tuple(float(x) for x in h)
        dim = len(self.shape)
        if dim not in (2, 3) or len(self.h) != dim:
            raise ValueError("shape and h must both have length 2 or 3")
        if bc not in BCS:
            raise ValueError(f"unknown bc {bc!r}")
        self.bc = bc
        n = (ctypes.c_int64 * 3)(*(list(self.shape) + [1] * (3 - dim)))
        hh = (ctypes.c_double * 3)(*(list(self.h) + [1.0] * (3 - dim)))
        kind, c0, c1 = COEF_CONST, 1.0, 0.0
        tabs = [None, None, None]
        field = None
        if coef is None:
            pass
        elif isinstance(coef, (int, float)):
            c0 = float(coef)
        elif isinstance(coef, tuple) and coef and coef[0] == "dlap":
            kind = COEF_DLAP
            c0 = float(coef[1]) if len(coef) > 1 else 1.0
        elif isinstance(coef, tuple) and coef and coef[0] == "separable":
            kind = COEF_SEPARABLE
            c0, c1 = float(coef[1]), float(coef[2])
            for d in range(dim):
                t = _dev_f64(coef[3 + d], self.device, self.shape[d], f"table {d}")
                self._keep.append(t)
                tabs[d] = t
        else:
            kind = COEF_FIELD
            field = _dev_f64(coef, self.device, int(torch.tensor(self.shape).prod()), "field")
            self._keep.append(field)
        self.coef_kind = kind
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        with torch.cuda.device(self.device):
            check(lib().expi_op_create_stencil(ctypes.byref(self._h), dim, n, hh, BCS[bc], kind,
                                               c0, c1, ptr(tabs[0]), ptr(tabs[1]), ptr(tabs[2]),
                                               ptr(field)))


    def set_boundary_data(self, kind, mode: str = "in_kernel") -> None:
        """Inhomogeneous Dirichlet data (3D dirichlet0): kind 'z1mz_xy',
        'sinpiz_expmxy' or None; mode 'in_kernel' or 'separate'
        (expi_op_set_boundary_data)."""
        if kind not in BDATA or mode not in BDATA_MODES:
            raise ValueError(f"boundary data {kind!r} / mode {mode!r} unknown")
        check(lib().expi_op_set_boundary_data(self._h, BDATA[kind], BDATA_MODES[mode]))


class CsrOp(_Op):
    """CSR matrix, int32 row pointers/column indices and float64 values."""

    def __init__(self, n, rowptr, colind, val, device="cuda:0"):
        super().__init__()
        torch = _torch()
        self.device = torch.device(device)
        rp = torch.as_tensor(rowptr).to(device=self.device, dtype=torch.int32).contiguous()
        ci = torch.as_tensor(colind).to(device=self.device, dtype=torch.int32).contiguous()
        va = _dev_f64(val, self.device)
        if rp.numel() != n + 1 or ci.numel() != va.numel():
            raise ValueError("inconsistent CSR array sizes")
        self._keep += [rp, ci, va]
        self.nnz = int(va.numel())
        check(lib().expi_op_create_csr(ctypes.byref(self._h), int(n), self.nnz,
                                       ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                                       ctypes.c_void_p(va.data_ptr())))


class CsrComplexOp(_Op):
    """Hermitian CSR matrix with complex128 values (int32 indices); vectors
    are complex128 tensors (stored as (re, im) float64 pairs)."""

    def __init__(self, n, rowptr, colind, val, device="cuda:0"):
        super().__init__()
        torch = _torch()
        self.device = torch.device(device)
        rp = torch.as_tensor(rowptr).to(device=self.device, dtype=torch.int32).contiguous()
        ci = torch.as_tensor(colind).to(device=self.device, dtype=torch.int32).contiguous()
        va = torch.as_tensor(val).to(device=self.device, dtype=torch.complex128).contiguous()
        if rp.numel() != n + 1 or ci.numel() != va.numel():
            raise ValueError("inconsistent CSR array sizes")
        self._keep += [rp, ci, va]
        self.nnz = int(va.numel())
        check(lib().expi_op_create_csr_complex(ctypes.byref(self._h), int(n), self.nnz,
                                               ctypes.c_void_p(rp.data_ptr()),
                                               ctypes.c_void_p(ci.data_ptr()),
                                               ctypes.c_void_p(va.data_ptr())))


def skew_phi_action(op: CsrComplexOp, k: int, tau: float, v, y=None, tol: float = 1e-10,
                    params: LejaParams | None = None, ws=None, stream=None):
    """y = phi_k(-i tau H) v (k = 0 or 1) for a Hermitian complex CSR operator;
    v complex128 on the op's device.  Returns (y, stats dict)."""
    torch = _torch()
    if v.dtype != torch.complex128:
        raise ValueError("v must be complex128")
    if y is None:
        y = torch.empty_like(v)
    if ws is None:
        ws = op.workspace("f64")
    st = Stats()
    cp = params.to_c() if params is not None else None
    check(lib().expi_skew_phi_action(op.handle, int(k), float(tau), ctypes.c_void_p(v.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()), float(tol),
                                     ctypes.byref(cp) if cp is not None else None,
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(st),
                                     _stream_ptr(stream, op.device)))
    return y, st.as_dict()


def workspace(nbytes: int, device="cuda:0"):
    """Device byte buffer, 256-byte aligned, for phi_action/expeuler_step."""
    torch = _torch()
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


def apply_op(op: _Op, alpha: float, beta: float, x, y=None, stream=None):
    """y = (alpha A + beta I) x (eq. (3)); x float64 or float32 on the op's device."""
    torch = _torch()
    code = F32 if x.dtype == torch.float32 else F64     # complex128 is F64 pairs
    if y is None:
        y = torch.empty_like(x)
    check(lib().apply_op(op.handle, float(alpha), float(beta), ctypes.c_void_p(x.data_ptr()),
                         ctypes.c_void_p(y.data_ptr()), code, _stream_ptr(stream, op.device)))
    return y


def phi_action(op: _Op, k: int, tau: float, v, y=None, tol: float = 1e-10, dtype="f64",
               params: LejaParams | None = None, ws=None, stream=None):
    """y = phi_k(tau A) v; returns (y, stats dict)."""
    torch = _torch()
    if y is None:
        y = torch.empty_like(v)
    code = _dtype_code(dtype)
    if ws is None:
        ws = op.workspace(code)
    st = Stats()
    cp = params.to_c() if params is not None else None
    rc = lib().phi_action(op.handle, int(k), float(tau), ctypes.c_void_p(v.data_ptr()),
                          ctypes.c_void_p(y.data_ptr()), float(tol), code,
                          ctypes.byref(cp) if cp is not None else None,
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(st),
                          _stream_ptr(stream, op.device))
    check(rc)
    return y, st.as_dict()


def noalloc_init(device="cuda:0") -> None:
    """Set-up of phi_action_noalloc for this thread and device (expi_noalloc_init)."""
    torch = _torch()
    with torch.cuda.device(torch.device(device)):
        check(lib().expi_noalloc_init())


def phi_action_noalloc(op: _Op, k: int, tau: float, v, y, tol: float = 1e-10, dtype="f64",
                       params: LejaParams | None = None, stream=None):
    """y = phi_k(tau A) v with the library's scratch array as workspace (no
    device allocation in the call; y must be given); returns the stats dict."""
    torch = _torch()
    st = Stats()
    cp = params.to_c() if params is not None else None
    with torch.cuda.device(op.device):
        rc = lib().phi_action_noalloc(op.handle, int(k), float(tau), ctypes.c_void_p(v.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), float(tol), _dtype_code(dtype),
                                      ctypes.byref(cp) if cp is not None else None,
                                      ctypes.byref(st), _stream_ptr(stream, op.device))
    check(rc)
    return st.as_dict()


def _nonlin_code(g) -> int:
    if g not in NONLIN:
        raise ValueError(f"nonlinearity must be one of {sorted(NONLIN)}, got {g!r}")
    return NONLIN[g]


def expeuler_step(op: _Op, tau: float, u, tol: float = 1e-10, dtype="f64",
                  params: LejaParams | None = None, ws=None, stream=None, g="cubic"):
    """One exponential Euler step for u' = A u + g(u), in place on u; g is
    'cubic' (u - u^3), 'combustion' or 'combustion_fast'; returns stats."""
    code = _dtype_code(dtype)
    if ws is None:
        ws = op.workspace(code)
    st = Stats()
    cp = params.to_c() if params is not None else None
    rc = lib().expeuler_step(op.handle, _nonlin_code(g), float(tau), ctypes.c_void_p(u.data_ptr()),
                             float(tol), code, ctypes.byref(cp) if cp is not None else None,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(st),
                             _stream_ptr(stream, op.device))
    check(rc)
    return st.as_dict()


def exprk2_step(op: _Op, tau: float, u, tol: float = 1e-10, dtype="f64",
                params: LejaParams | None = None, ws=None, stream=None, g="cubic"):
    """One step of the second-order exponential Runge-Kutta method (exprk2_step),
    in place on u; returns stats."""
    code = _dtype_code(dtype)
    if ws is None:
        key = ("rk2", code)
        ws = op._ws.get(key)
        if ws is None:
            ws = workspace(int(lib().expi_exprk2_workspace_bytes(op.handle, code)), op.device)
            op._ws[key] = ws
    st = Stats()
    cp = params.to_c() if params is not None else None
    rc = lib().exprk2_step(op.handle, _nonlin_code(g), float(tau), ctypes.c_void_p(u.data_ptr()),
                           float(tol), code, ctypes.byref(cp) if cp is not None else None,
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(st),
                           _stream_ptr(stream, op.device))
    check(rc)
    return st.as_dict()


def nonlinearity(g: str, u, out=None, stream=None):
    """out = g(u) pointwise on the device (expi_nonlinearity); u float64 or float32."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(u)
    code = F32 if u.dtype == torch.float32 else F64
    check(lib().expi_nonlinearity(_nonlin_code(g), u.numel(), ctypes.c_void_p(u.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), code,
                                  _stream_ptr(stream, u.device)))
    return out


class Batch:
    """Many independent 2D problems y_i = phi_1(tau_i A_i) v_i solved together
    in rounds of two kernels each (expi_batch_*), eagerly or as a replayed
    HIP graph.  A_i = coef * 5-point Laplacian on an nx_i x ny_i grid with
    spacing (hx_i, hy_i) and boundary `bc`.  Vectors are concatenated;
    `offsets[i]` is where instance i starts."""

    def __init__(self, nx, ny, hx, hy, tau, bc="dirichlet0", coef=1.0, tol=1e-8, dtype="f32",
                 params: LejaParams | None = None, device="cuda:0"):
        import numpy as np
        torch = _torch()
        self.device = torch.device(device)
        self.count = len(nx)
        arr = lambda a, t: np.ascontiguousarray(np.asarray(a, dtype=t))
        self._nx, self._ny = arr(nx, np.int32), arr(ny, np.int32)
        self._hx, self._hy, self._tau = arr(hx, np.float64), arr(hy, np.float64), arr(tau, np.float64)
        for a_ in (self._ny, self._hx, self._hy, self._tau):
            if a_.size != self.count:
                raise ValueError("per-instance arrays differ in length")
        if bc not in ("dirichlet0", "neumann0"):
            raise ValueError("bc must be dirichlet0 or neumann0")
        self.bc, self.dtype = bc, dtype
        self._h = ctypes.c_void_p()
        cp = params.to_c() if params is not None else None
        i32 = ctypes.POINTER(ctypes.c_int32)
        dbl = ctypes.POINTER(ctypes.c_double)
        check(lib().expi_batch_create(ctypes.byref(self._h), self.count,
                                      self._nx.ctypes.data_as(i32), self._ny.ctypes.data_as(i32),
                                      self._hx.ctypes.data_as(dbl), self._hy.ctypes.data_as(dbl),
                                      self._tau.ctypes.data_as(dbl), BCS[bc], float(coef),
                                      float(tol), _dtype_code(dtype),
                                      ctypes.byref(cp) if cp is not None else None))
        self.total_length = int(lib().expi_batch_total_length(self._h))
        off = np.zeros(self.count, dtype=np.int64)
        check(lib().expi_batch_offsets(self._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        self.offsets = off
        self._ws = None

    @property
    def handle(self):
        return self._h

    def sizes(self):
        return [(int(a), int(b)) for a, b in zip(self._nx, self._ny)]

    def workspace(self):
        if self._ws is None:
            self._ws = workspace(int(lib().expi_batch_workspace_bytes(self._h)), self.device)
        return self._ws

    def tiles(self):
        w, m = ctypes.c_int(), ctypes.c_int()
        check(lib().expi_batch_get_tiles(self._h, ctypes.byref(w), ctypes.byref(m)))
        return (w.value, m.value)

    @property
    def pairs(self) -> bool:
        """Newton products two per round (the default) or one."""
        on = ctypes.c_int()
        check(lib().expi_batch_get_pairs(self._h, ctypes.byref(on)))
        return bool(on.value)

    def set_pairs(self, on: bool) -> None:
        check(lib().expi_batch_set_pairs(self._h, int(bool(on))))

    def set_tiles(self, waves: int, march: int) -> None:
        check(lib().expi_batch_set_tiles(self._h, int(waves), int(march)))
        nb = int(lib().expi_batch_workspace_bytes(self._h))
        if self._ws is not None and self._ws.numel() < nb:
            self._ws = None

    def prepare(self, stream=None):
        ws = self.workspace()
        check(lib().expi_batch_prepare(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_ptr(stream, self.device)))

    def _run_args(self, v, y):
        ws = self.workspace()
        return (self._h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                ctypes.c_void_p(ws.data_ptr()), ws.numel())

    def launch(self, v, y, stream=None):
        """Solve every instance (returns once the device is done)."""
        check(lib().expi_batch_launch(*self._run_args(v, y), _stream_ptr(stream, self.device)))

    def capture(self, v, y, rounds: int = 0, stream=None):
        """Record reset + `rounds` rounds (0: enough for every instance) as a graph."""
        check(lib().expi_batch_capture(*self._run_args(v, y), int(rounds),
                                       _stream_ptr(stream, self.device)))

    def replay(self, stream=None):
        check(lib().expi_batch_replay(self._h, _stream_ptr(stream, self.device)))

    @property
    def max_rounds(self) -> int:
        return int(lib().expi_batch_max_rounds(self._h))

    @property
    def graph_rounds(self) -> int:
        return int(lib().expi_batch_graph_rounds(self._h))

    def launch_persistent(self, v, y, stream=None):
        """All rounds in one persistent (cooperative) kernel launch."""
        check(lib().expi_batch_launch_persistent(*self._run_args(v, y),
                                                 _stream_ptr(stream, self.device)))

    def capture_persistent(self, v, y, stream=None):
        check(lib().expi_batch_capture_persistent(*self._run_args(v, y),
                                                  _stream_ptr(stream, self.device)))

    def results(self, stream=None, check_status=True):
        """(per-instance stat dicts, rounds); raises on failure if check_status."""
        st = (BatchStat * self.count)()
        rounds = ctypes.c_int()
        ws = self.workspace()
        rc = lib().expi_batch_results(self._h, ctypes.c_void_p(ws.data_ptr()),
                                      _stream_ptr(stream, self.device), st, ctypes.byref(rounds))
        if check_status:
            check(rc)
        return [s.as_dict() for s in st], rounds.value

    def __del__(self):
        try:
            if self._h:
                lib().expi_batch_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass
