"""Host-side tests of libexpi.so that need no GPU.

* the library loads and exports every function include/expi.h declares;
* its Leja points and divided differences (long double, written separately
  from the oracle's mpmath code) agree with the oracle;
* argument validation returns the documented codes before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import leja as oleja

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1309_4616_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_1309_4616_amd import build
        build.build()
    return _binding.lib()


def header_functions():
    text = open(os.path.join(ROOT, "include", "expi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_exports_every_declared_function(L):
    names = header_functions()
    assert {"apply_op", "phi_action", "expeuler_step"} <= set(names)
    for name in names:
        assert hasattr(L, name), name
    from paper_1309_4616_amd import _binding
    assert set(_binding.EXPORTS) == set(names)


def test_leja_points_match_oracle(L):
    from paper_1309_4616_amd import _binding
    lib_pts = _binding.leja_points(256)
    ora = oleja.leja_points(256)
    assert np.max(np.abs(lib_pts - ora)) <= 2e-15
    assert lib_pts[0] == 2.0 and lib_pts[1] == -2.0


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("length", [0.5, 13.3, 60.0, 100.0])
def test_divided_differences_match_oracle(L, k, length):
    """The two sets of differences define the same interpolant on [-2, 2]
    (individual tail differences are below rounding of the leading ones)."""
    from paper_1309_4616_amd import _binding
    c, gamma = -length / 2, length / 4
    xi = oleja.leja_points(101)
    d_lib = _binding.divided_differences(k, 1.0, c, gamma, 101)
    d_or = oleja.divided_differences(k, 1.0, c, gamma, xi)
    grid = np.linspace(-2, 2, 2001)
    diff = np.max(np.abs(oleja.newton_eval(d_lib, xi, grid) - oleja.newton_eval(d_or, xi, grid)))
    assert diff <= 1e-14
    lead = np.abs(d_or) > 1e-8 * np.abs(d_or).max()
    assert np.allclose(d_lib[lead], d_or[lead], rtol=1e-9, atol=0)


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("length", [3.0, 40.0, 100.0])
def test_skew_divided_differences_match_oracle(L, k, length):
    """The complex coefficients of phi_k(-i delta H) (long double in the
    library, 80-digit mpmath in the oracle) define the same interpolant."""
    from paper_1309_4616_amd import _binding
    c, gamma = 7.0, length / 4
    xi = oleja.leja_points(101)
    lib_d = _binding.divided_differences_skew(k, 1.0, c, gamma, 101)
    ora_d = oleja.divided_differences_skew(k, 1.0, c, gamma, xi)
    xs = np.linspace(-2, 2, 801)

    def newton(d):
        p = np.zeros(xs.shape, dtype=np.complex128)
        w = np.ones(xs.shape)
        for j in range(len(d)):
            p += d[j] * w
            w = w * (xs - xi[j])
        return p
    pl, po = newton(lib_d), newton(ora_d)
    assert np.max(np.abs(pl - po)) <= 1e-13 * max(1.0, np.max(np.abs(po)))


def _stencil(L, dim=2, n=(8, 8, 8), h=(0.1, 0.1, 0.1), bc=0, kind=0, tabs=(None, None, None), field=None):
    op = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 3)(*n)
    hh = (ctypes.c_double * 3)(*h)
    rc = L.expi_op_create_stencil(ctypes.byref(op), dim, nn, hh, bc, kind, 1.0, 0.5,
                                  tabs[0], tabs[1], tabs[2], field)
    return rc, op


def test_create_validation(L):
    assert _stencil(L, dim=1)[0] == -1
    assert _stencil(L, dim=4)[0] == -1
    assert _stencil(L, n=(0, 4, 4))[0] == -1
    assert _stencil(L, h=(0.1, -1.0, 0.1))[0] == -1
    assert _stencil(L, bc=7)[0] == -1
    assert _stencil(L, kind=1)[0] == -1          # separable without tables
    assert _stencil(L, kind=2)[0] == -1          # field without array
    assert _stencil(L, kind=9)[0] == -1
    assert _stencil(L, dim=3, n=(1024, 1024, 1024))[0] == -1   # 2^30 points
    rc, op = _stencil(L, dim=3, n=(5, 6, 7))
    assert rc == 0 and L.expi_op_size(op) == 210
    assert L.expi_workspace_bytes(op, 0) > L.expi_workspace_bytes(op, 1) > 0
    assert L.expi_workspace_bytes(op, 5) == 0
    L.expi_op_destroy(op)
    op2 = ctypes.c_void_p()
    assert L.expi_op_create_csr(ctypes.byref(op2), 0, 0, None, None, None) == -1
    assert L.expi_op_create_csr(ctypes.byref(op2), 10, 5, None, None, None) == -1


def test_call_validation_before_any_hip_call(L):
    from paper_1309_4616_amd import _binding
    rc, op = _stencil(L, dim=2, n=(16, 16, 1))
    assert rc == 0
    need = L.expi_workspace_bytes(op, 0)
    buf = ctypes.create_string_buffer(need + 512)
    base = ctypes.addressof(buf)
    ws = ctypes.c_void_p((base + 255) & ~255)
    v = ctypes.create_string_buffer(16 * 16 * 8)
    y = ctypes.create_string_buffer(16 * 16 * 8)
    st = _binding.Stats()
    vp, yp = ctypes.c_void_p(ctypes.addressof(v)), ctypes.c_void_p(ctypes.addressof(y))
    call = lambda **kw: L.phi_action(kw.get("op", op), kw.get("k", 1), kw.get("tau", 1e-3),
                                     kw.get("v", vp), kw.get("y", yp), kw.get("tol", 1e-10),
                                     kw.get("dtype", 0), kw.get("params", None), kw.get("ws", ws),
                                     kw.get("wsb", need), ctypes.byref(st), None)
    assert call(op=None) == -1
    assert call(tau=-1.0) == -1
    assert call(tau=float("nan")) == -1
    assert call(tol=0.0) == -1
    assert call(dtype=3) == -1
    assert call(k=-1) == -1
    assert call(v=None) == -1
    assert call(y=vp) == -2                        # y aliases v
    assert call(ws=None) == -3
    assert call(wsb=need - 1) == -3
    assert call(ws=ctypes.c_void_p(ws.value + 8)) == -3   # misaligned
    bad = _binding.LejaParams(m_max=1).to_c()
    assert call(params=ctypes.byref(bad)) == -1
    bad = _binding.LejaParams(m_max=256).to_c()
    assert call(params=ctypes.byref(bad)) == -1
    bad = _binding.LejaParams(interval=(0.0, -1.0)).to_c()
    assert call(params=ctypes.byref(bad)) == -1
    assert b"interval" in L.expi_last_error()
    bad = _binding.LejaParams(fuse_start=3).to_c()
    assert call(params=ctypes.byref(bad)) == -1
    assert b"fuse_start" in L.expi_last_error()
    x = ctypes.c_void_p(ctypes.addressof(v))
    assert L.apply_op(op, 1.0, 0.0, x, x, 0, None) == -2
    assert L.apply_op(op, float("inf"), 0.0, x, yp, 0, None) == -1
    assert L.expeuler_step(op, 7, 1e-3, yp, 1e-10, 0, None, ws, need, ctypes.byref(st), None) == -1
    assert b"nonlin" in L.expi_last_error()
    # the second-order step needs one more float64 vector of workspace
    need2 = L.expi_exprk2_workspace_bytes(op, 0)
    assert need2 >= need + 16 * 16 * 8
    assert L.exprk2_step(op, 0, 1e-3, yp, 1e-10, 0, None, ws, need, ctypes.byref(st), None) == -3
    assert L.exprk2_step(op, 3, 1e-3, yp, 1e-10, 0, None, ws, need, ctypes.byref(st), None) == -1
    assert L.exprk2_step(op, 0, -1.0, yp, 1e-10, 0, None, ws, need, ctypes.byref(st), None) == -1
    # the pointwise nonlinearity kernel
    assert L.expi_nonlinearity(5, 16, vp, yp, 0, None) == -1
    assert L.expi_nonlinearity(1, 16, vp, yp, 2, None) == -1
    assert L.expi_nonlinearity(1, -1, vp, yp, 0, None) == -1
    assert L.expi_nonlinearity(1, 0, None, None, 0, None) == 0
    assert L.expi_nonlinearity(1, 16, vp, ctypes.c_void_p(ctypes.addressof(v) + 8), 0, None) == -2
    nc = ctypes.c_int()
    assert L.expi_op_autotune(op, 0, 0, ws, need, None, None, None, 0, ctypes.byref(nc)) == -1
    assert L.expi_op_autotune(op, 0, 5, ws, need - 1, None, None, None, 0, ctypes.byref(nc)) == -3
    assert L.expi_op_set_tiles(op, 3, 4, 8) == -1
    assert L.expi_op_set_tiles(op, 2, 9, 8) == -1
    assert L.expi_op_set_tiles(op, 2, 4, 6) == -1
    assert L.expi_op_set_tiles(op, 1, 2, 16) == 0
    v_, w_, m_ = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.expi_op_get_tiles(op, ctypes.byref(v_), ctypes.byref(w_), ctypes.byref(m_)) == 0
    assert (v_.value, w_.value, m_.value) == (1, 2, 16)
    use = ctypes.c_int()
    assert L.expi_op_get_pairs(op, ctypes.byref(use)) == 0 and use.value == 1
    assert L.expi_op_set_pairs(op, 2) == -1
    assert L.expi_op_set_pairs(op, 0) == 0
    assert L.expi_op_get_pairs(op, ctypes.byref(use)) == 0 and use.value == 0
    L.expi_op_destroy(op)


def test_pair_rows_setting(L):
    """A 2D constant-coefficient operator with pair sweeps also takes a tile
    height for them (a multiple of 4 up to 64); other operators take only
    0 or 1."""
    use = ctypes.c_int()
    rc, op2 = _stencil(L, dim=2, bc=0)
    assert rc == 0
    for bad in (2, 3, 30, 68, -4):
        assert L.expi_op_set_pairs(op2, bad) == -1
    for good in (4, 32, 64, 1, 0):
        assert L.expi_op_set_pairs(op2, good) == 0
        assert L.expi_op_get_pairs(op2, ctypes.byref(use)) == 0 and use.value == good
    L.expi_op_destroy(op2)
    rc, op = _stencil(L, dim=2, bc=2)    # only the interior rows: a 2D pair sweep too
    assert rc == 0 and L.expi_op_set_pairs(op, 32) == 0
    L.expi_op_destroy(op)
    rc, op = _stencil(L, dim=3, bc=0)    # a 3D operator: on or off only
    assert rc == 0
    assert L.expi_op_set_pairs(op, 32) == -1
    assert L.expi_op_set_pairs(op, 1) == 0
    L.expi_op_destroy(op)


def test_noalloc_size_limit_before_any_hip_call(L):
    """The allocation-free phi_action refuses an operator whose workspace is
    larger than the library's scratch array, and a bad dtype, before it
    touches the device."""
    from paper_1309_4616_amd import _binding
    rc, op = _stencil(L, dim=3, n=(256, 256, 256))
    assert rc == 0
    assert L.expi_workspace_bytes(op, 0) > _binding.NOALLOC_SCRATCH_BYTES
    st = _binding.Stats()
    v = ctypes.c_void_p(1 << 20)
    y = ctypes.c_void_p(1 << 32)
    assert L.phi_action_noalloc(op, 1, 1e-5, v, y, 1e-10, 0, None, ctypes.byref(st), None) == -3
    assert b"scratch" in L.expi_last_error()
    assert L.phi_action_noalloc(op, 1, 1e-5, v, y, 1e-10, 7, None, ctypes.byref(st), None) == -1
    assert L.phi_action_noalloc(None, 1, 1e-5, v, y, 1e-10, 0, None, ctypes.byref(st), None) == -1
    L.expi_op_destroy(op)


def test_batch_create_validation_and_layout(L):
    """The batch is built on the host (intervals, substeps, divided
    differences, offsets); no GPU is touched until prepare/launch."""
    import numpy as np
    from paper_1309_4616_amd import _binding
    nx = np.array([64, 33, 100], dtype=np.int32)
    ny = np.array([64, 40, 7], dtype=np.int32)
    h = 1.0 / (nx + 1.0)
    tau = np.array([1e-4, 2e-3, 0.0])
    i32 = ctypes.POINTER(ctypes.c_int32)
    dbl = ctypes.POINTER(ctypes.c_double)
    b = ctypes.c_void_p()
    args = lambda **kw: (ctypes.byref(b), kw.get("count", 3), nx.ctypes.data_as(i32), ny.ctypes.data_as(i32),
                         h.ctypes.data_as(dbl), h.ctypes.data_as(dbl), kw.get("tau", tau).ctypes.data_as(dbl),
                         kw.get("bc", 0), kw.get("coef", 1.0), kw.get("tol", 1e-8), kw.get("dtype", 1), None)
    assert L.expi_batch_create(*args(count=0)) == -1
    assert L.expi_batch_create(*args(bc=2)) == -1
    assert L.expi_batch_create(*args(coef=0.0)) == -1
    assert L.expi_batch_create(*args(tol=-1.0)) == -1
    assert L.expi_batch_create(*args(tau=np.array([1e-4, -1.0, 0.0]))) == -1
    assert L.expi_batch_create(*args()) == 0
    total = L.expi_batch_total_length(b)
    off = np.zeros(3, dtype=np.int64)
    assert L.expi_batch_offsets(b, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))) == 0
    assert off[0] == 0 and np.all(off % 32 == 0)
    assert np.all(np.diff(off) >= (nx * ny)[:-1]) and total >= off[-1] + nx[-1] * ny[-1]
    ws_bytes = L.expi_batch_workspace_bytes(b)
    assert ws_bytes > 3 * 4 * total
    assert L.expi_batch_set_tiles(b, 9, 8) == -1
    assert L.expi_batch_set_tiles(b, 2, 6) == -1
    assert L.expi_batch_set_tiles(b, 2, 16) == 0
    assert L.expi_batch_workspace_bytes(b) == ws_bytes
    on = ctypes.c_int(-1)
    assert L.expi_batch_get_pairs(b, ctypes.byref(on)) == 0 and on.value == 1   # two products per round by default
    assert L.expi_batch_set_pairs(b, 2) == -1
    assert L.expi_batch_set_pairs(None, 0) == -1
    assert L.expi_batch_get_pairs(b, None) == -1
    assert L.expi_batch_set_pairs(b, 0) == 0
    assert L.expi_batch_get_pairs(b, ctypes.byref(on)) == 0 and on.value == 0
    assert L.expi_batch_set_pairs(b, 1) == 0
    # substeps from the closed-form interval: s_i = ceil(tau_i 4 (2/h_i^2) / 100)
    s_want = np.maximum(np.ceil(tau * 8.0 / h**2 / 100.0), 1).astype(int)
    assert L.expi_batch_max_rounds(b) == int(s_want.max()) * (100 + 2) + 2
    assert L.expi_batch_graph_rounds(b) == 0
    assert L.expi_batch_launch(b, None, None, None, 0, None) == -1
    assert L.expi_batch_replay(b, None) == -1        # nothing captured
    dummy = ctypes.c_void_p(256)
    # launching or capturing needs a prepared workspace (checked before any HIP call)
    assert L.expi_batch_launch(b, dummy, ctypes.c_void_p(1 << 40), dummy, ws_bytes, None) == -1
    assert b"prepare" in L.expi_last_error()
    assert L.expi_batch_capture(b, dummy, ctypes.c_void_p(1 << 40), dummy, ws_bytes, 0, None) == -1
    # so does the persistent launch
    assert L.expi_batch_launch_persistent(b, dummy, ctypes.c_void_p(1 << 40), dummy, ws_bytes, None) == -1
    assert b"prepare" in L.expi_last_error()
    assert L.expi_batch_capture_persistent(b, dummy, ctypes.c_void_p(1 << 40), dummy, ws_bytes, None) == -1
    L.expi_batch_destroy(b)
