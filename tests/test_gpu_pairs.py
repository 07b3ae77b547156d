"""GPU parity of the pair sweep (two Newton products per pass).

phi_1(tau A) v on 3D stencils with the pair sweep on (the default where it
applies) against the FP64 oracle, over shapes that exercise its tiling: one
and two waves per row, rows ragged against the row tile, few planes,
chunks that cross row tiles, every boundary handling, both coefficient kinds
it covers, FP32 storage, and stops after either product of a pair (the
second case removes the extra term).  The single-product path on the same
inputs must agree.
"""
import math

import numpy as np
import pytest

import synth
from oracle import integrators as I
from oracle import operators as O

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10


@pytest.fixture(scope="module")
def E(device):
    import paper_1309_4616_amd as E
    E.lib()
    return E


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make(E, shape, bc, kind):
    h = tuple(1.0 / s for s in shape)
    if kind == "const":
        return E.StencilOp(shape, h, bc, coef=1.3), O.stencil_matrix(shape, h, bc, coef=1.3)
    tabs = [np.cos(2 * math.pi * (np.arange(s) + 0.5) / s) for s in shape]
    c0, c1 = 1.0, 0.45
    fld = c0 + c1 * ((tabs[2][:, None, None] * tabs[1][None, :, None]) * tabs[0][None, None, :])
    op = E.StencilOp(shape, h, bc, coef=("separable", c0, c1, *tabs))
    return op, O.stencil_matrix(shape, h, bc, coef=fld.reshape(-1))


def run_pair_and_single(E, op, v, tau, tol, dtype="f64", interval=None):
    yp, sp = E.phi_action(op, 1, tau, T(v), tol=tol, dtype=dtype,
                          params=E.LejaParams(profile=True, interval=interval))
    ys, ss = E.phi_action(op, 1, tau, T(v), tol=tol, dtype=dtype,
                          params=E.LejaParams(pairs=False, profile=True, interval=interval))
    return N(yp), sp, N(ys), ss


SHAPES = [
    (256, 12, 9),     # two waves per row, rows ragged against the 6-row tile
    (128, 20, 7),     # one wave per row, 14-row tiles
    (130, 7, 5),      # two waves, second nearly empty
    (64, 6, 33),      # many planes: chunks cross row tiles
    (2, 3, 4),        # tiny
    (200, 1, 3),      # a single row
    (96, 15, 1),      # a single plane
    (512, 7, 6),      # four waves per row, 2-row tiles, ragged rows
    (300, 5, 8),      # four waves per row, the last one beyond the row end
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
def test_pair_sweep_phi1_matches_oracle(E, shape, bc):
    for kind in ("const", "separable"):
        op, A = make(E, shape, bc, kind)
        n = int(np.prod(shape))
        v = synth.uniform_vector(n, 7)
        a, b = O.gershgorin_interval(A)
        # interior_only with a side of at most 2 points has no interior: A = 0
        # and a = b, so both sides get the interval [-1, 0] instead
        iv = None if b > a else (-1.0, 0.0)
        tau = 8.0 / (b - a) if iv is None else 1e-3     # tau (b - a) = 8: one substep
        print(f"pair phi1 {shape} {bc} {kind}", flush=True)
        yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-10, interval=iv)
        yo, so = I.phi_action(A, 1, tau, v, 1e-10, interval=iv)
        assert relerr(yp, yo) <= TOL_F64, (kind, relerr(yp, yo))
        assert relerr(ys, yo) <= TOL_F64
        assert abs(sp["degree_last"] - so.degrees[-1]) <= 1
        # the pair path took pair sweeps (it applies to every shape here);
        # the pair over products 0 and 1 is not timed, so a stop at m = 2
        # shows none
        assert sp["degree_last"] <= 2 or sp["timed_pairs"] >= 1
        assert ss["timed_pairs"] == 0


def test_pair_stops_after_either_product(E):
    """Vary tau so the stop falls after the first and after the second
    product of a pair; both match the oracle, the first with the extra term
    removed."""
    shape = (256, 10, 6)
    op, A = make(E, shape, "neumann0", "separable")
    n = int(np.prod(shape))
    v = synth.uniform_vector(n, 3)
    a, b = O.gershgorin_interval(A)
    parities = set()
    for q in np.linspace(2.0, 40.0, 12):
        tau = q / (b - a)
        yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-10)
        yo, so = I.phi_action(A, 1, tau, v, 1e-10)
        assert relerr(yp, yo) <= TOL_F64, (q, relerr(yp, yo))
        assert sp["degree_last"] == ss["degree_last"]
        parities.add(sp["degree_last"] % 2)
    assert parities == {0, 1}


def test_pair_substeps_expeuler_and_fp32(E):
    """Several substeps (start vectors between loops), the exponential Euler
    step, and FP32 storage through the pair sweep."""
    shape = (256, 14, 11)
    op, A = make(E, shape, "neumann0", "separable")
    n = int(np.prod(shape))
    v = synth.uniform_vector(n, 5)
    a, b = O.gershgorin_interval(A)
    tau = 230.0 / (b - a)                      # three substeps
    yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-10)
    yo, so = I.phi_action(A, 1, tau, v, 1e-10)
    assert sp["substeps"] == so.substeps == 3
    assert relerr(yp, yo) <= TOL_F64 and relerr(ys, yo) <= TOL_F64
    y32, s32 = E.phi_action(op, 1, tau, T(v), tol=1e-10, dtype="f32")
    assert relerr(N(y32), yo) <= 5e-6
    u0 = 0.5 + 0.1 * synth.uniform_vector(n, 9)
    tau_e = 20.0 / (b - a)
    u = T(u0)
    st = E.expeuler_step(op, tau_e, u, tol=1e-10)
    uo, _ = I.expeuler_step(A, tau_e, u0, 1e-10)
    assert relerr(N(u), uo) <= TOL_F64
    assert st["converged"] == 1


def test_pair_profile_accounting(E):
    shape = (256, 30, 20)
    op, A = make(E, shape, "dirichlet0", "const")
    v = synth.uniform_vector(int(np.prod(shape)), 1)
    a, b = O.gershgorin_interval(A)
    yp, sp, ys, ss = run_pair_and_single(E, op, v, 30.0 / (b - a), 1e-10)
    m = sp["degree_last"]
    # first product single, then pairs (and maybe one single) up to the stop
    assert sp["timed_products"] >= m - 1 - 1 and sp["timed_products"] <= m
    assert sp["timed_pairs"] >= (m - 2) // 2 - 1
    assert 0 < sp["pair_ms"] <= sp["newton_ms"]
    assert ss["timed_products"] == m - 1 and ss["timed_pairs"] == 0
    # launches that did work: products 0 .. m-1 (a pair may end one past m)
    assert 2 * sp["pair_launches"] + sp["single_launches"] in (m, m + 1)
    assert ss["single_launches"] == m and ss["pair_launches"] == 0
    # profile = 2 times only the first launch after the opening pair sweep
    y2, s2 = E.phi_action(op, 1, 30.0 / (b - a), T(v), tol=1e-10, params=E.LejaParams(profile=2))
    assert s2["timed_pairs"] == 1 and s2["timed_products"] == 2 and s2["pair_ms"] > 0
    assert np.max(np.abs(N(y2) - yp)) <= 1e-12 * np.max(np.abs(yp))


def test_pair_fp32_constant_coefficient(E):
    """FP32 storage takes pair sweeps for both coefficient kinds."""
    shape = (256, 9, 13)
    op, A = make(E, shape, "dirichlet0", "const")
    v = synth.uniform_vector(int(np.prod(shape)), 2)
    a, b = O.gershgorin_interval(A)
    tau = 25.0 / (b - a)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10, dtype="f32", params=E.LejaParams(profile=True))
    yo, _ = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(y), yo) <= 5e-6
    assert st["timed_pairs"] >= 1
    op2, A2 = make(E, shape, "dirichlet0", "separable")
    y2, st2 = E.phi_action(op2, 1, tau, T(v), tol=1e-10, dtype="f32", params=E.LejaParams(profile=True))
    yo2, _ = I.phi_action(A2, 1, tau, v, 1e-10)
    assert relerr(N(y2), yo2) <= 5e-6
    assert st2["timed_pairs"] >= 1


@pytest.mark.parametrize("shape", [(256, 12, 9), (128, 30, 5), (64, 7, 17), (512, 5, 9)])
def test_pair_equals_single_products_elementwise(E, shape):
    """Pair sweeps and single products give the same result to rounding at
    every point (a tighter check than the oracle bar: it would show a stale
    row or plane in the sweep's rings, e.g. at the first plane of a chunk)."""
    op, A = make(E, shape, "dirichlet0", "const")
    v = synth.uniform_vector(int(np.prod(shape)), 7)
    a, b = O.gershgorin_interval(A)
    for q in (2.0, 8.0, 30.0):
        yp, sp, ys, ss = run_pair_and_single(E, op, v, q / (b - a), 1e-13)
        assert sp["degree_last"] == ss["degree_last"]
        assert np.max(np.abs(yp - ys)) <= 1e-12 * np.max(np.abs(ys)), (shape, q)


def test_first_pair_and_its_fallbacks(E):
    """The loop opens with a pair sweep over products 0 and 1 when the start
    vector has the storage type and 16-byte alignment; a start vector at an
    8-byte offset, or FP64 input under FP32 storage, opens with a single
    product instead.  All agree with the oracle; tau = 0 stops at m = 2 in
    the first pair with y = v exactly."""
    import torch
    shape = (256, 11, 7)
    op, A = make(E, shape, "dirichlet0", "separable")
    n = int(np.prod(shape))
    v = synth.uniform_vector(n, 4)
    a, b = O.gershgorin_interval(A)
    for q in (3.0, 17.0):
        tau = q / (b - a)
        yo, so = I.phi_action(A, 1, tau, v, 1e-10)
        buf = torch.zeros(n + 1, dtype=torch.float64, device="cuda:0")
        buf[1:] = T(v)
        print(f"first pair q={q}", flush=True)
        y1, s1 = E.phi_action(op, 1, tau, buf[1:], tol=1e-10)   # 8-byte offset
        y2, s2 = E.phi_action(op, 1, tau, T(v), tol=1e-10)
        assert relerr(N(y1), yo) <= TOL_F64 and relerr(N(y2), yo) <= TOL_F64
        assert s1["degree_last"] == s2["degree_last"]
        assert np.max(np.abs(N(y1) - N(y2))) <= 1e-12 * np.max(np.abs(yo))
        y3, _ = E.phi_action(op, 1, tau, T(v), tol=1e-10, dtype="f32")
        assert relerr(N(y3), yo) <= 5e-6
    y0, s0 = E.phi_action(op, 1, 0.0, T(v), tol=1e-10)
    assert np.array_equal(N(y0), v)
    assert s0["degree_last"] == 2


@pytest.mark.parametrize("bc,kind", [("neumann0", "separable"), ("neumann0", "const"),
                                     ("dirichlet0", "const"), ("dirichlet0", "separable"),
                                     ("interior_only", "separable")])
def test_start_vector_fused_into_first_pair(E, bc, kind):
    """Euler steps whose start vector r = A u + u - u^3 is formed inside the
    first pair sweep (fuse_start = 2) agree with the oracle and, point by
    point, with the separate start sweep (fuse_start = 1), for stops at odd
    and even degrees; several substeps fuse only the first."""
    shape = (256, 10, 7)
    op, A = make(E, shape, bc, kind)
    n = int(np.prod(shape))
    u0 = 0.5 + 0.1 * synth.uniform_vector(n, 12)
    a, b = O.gershgorin_interval(A)
    degrees = set()
    for q in (3.0, 9.0, 21.0, 30.0, 230.0):
        tau = q / (b - a)
        uo, so = I.expeuler_step(A, tau, u0, 1e-10)
        got = {}
        for fs in (1, 2):
            u = T(u0)
            print(f"fused start {bc} {kind} q={q} fuse_start={fs}", flush=True)
            st = E.expeuler_step(op, tau, u, tol=1e-10, params=E.LejaParams(fuse_start=fs))
            assert st["converged"] == 1
            assert relerr(N(u), uo) <= TOL_F64, (q, fs, relerr(N(u), uo))
            got[fs] = (N(u), st)
        assert got[1][1]["degree_last"] == got[2][1]["degree_last"]
        assert got[1][1]["matvecs"] == got[2][1]["matvecs"]
        assert got[1][1]["substeps"] == got[2][1]["substeps"] == so.substeps
        assert np.max(np.abs(got[1][0] - got[2][0])) <= 1e-12 * np.max(np.abs(uo))
        degrees.add(got[2][1]["degree_last"] % 2)
    assert degrees == {0, 1}


@pytest.mark.parametrize("bc,kind", [("neumann0", "separable"), ("dirichlet0", "const"),
                                     ("dirichlet0", "separable"), ("interior_only", "const")])
def test_start_vector_fused_into_first_pair_fp32(E, bc, kind):
    """FP32 storage: the fused start pair reads u in FP64 and forms r in FP64
    (as the separate start sweep does), rounds it to FP32 and runs product 0
    in FP32.  Fused and separate agree with the oracle to the FP32 bar of
    phi_1 (and so with each other to twice it); the fused run fuses."""
    shape = (256, 10, 7)
    op, A = make(E, shape, bc, kind)
    n = int(np.prod(shape))
    u0 = 0.5 + 0.1 * synth.uniform_vector(n, 13)
    a, b = O.gershgorin_interval(A)
    for q in (9.0, 21.0, 230.0):
        tau = q / (b - a)
        uo, so = I.expeuler_step(A, tau, u0, 1e-10)
        got = {}
        for fs in (1, 2):
            u = T(u0)
            print(f"fused start fp32 {bc} {kind} q={q} fuse_start={fs}", flush=True)
            st = E.expeuler_step(op, tau, u, tol=1e-10, dtype="f32", params=E.LejaParams(fuse_start=fs))
            assert st["converged"] == 1
            # the FP32 bar of phi_1 (w, p rounded to FP32 at every product;
            # up to 3 substeps of degree up to 60 here)
            assert relerr(N(u), uo) <= 5e-6, (q, fs, relerr(N(u), uo))
            assert st["fused_starts"] == (1 if fs == 2 else 0)
            got[fs] = N(u)
        # each within the bar of the oracle, so within twice it of each other
        assert relerr(got[2], got[1]) <= 1e-5, (q, relerr(got[2], got[1]))


def test_fused_start_by_degree_parity(E):
    """The automatic choice (fuse_start = 0) over a run of steps gives the
    same states as never fusing."""
    shape = (256, 12, 9)
    op, A = make(E, shape, "neumann0", "separable")
    n = int(np.prod(shape))
    a, b = O.gershgorin_interval(A)
    for q in (7.0, 12.0):
        tau = q / (b - a)
        ua, ub = T(0.5 + 0.1 * synth.uniform_vector(n, 2)), None
        ub = ua.clone()
        uo = N(ua).copy()
        for step in range(4):
            E.expeuler_step(op, tau, ua, tol=1e-10, params=E.LejaParams(fuse_start=0))
            E.expeuler_step(op, tau, ub, tol=1e-10, params=E.LejaParams(fuse_start=1))
            uo, _ = I.expeuler_step(A, tau, uo, 1e-10)
            assert np.max(np.abs(N(ua) - N(ub))) <= 1e-12 * np.max(np.abs(N(ub))), (q, step)
            assert relerr(N(ua), uo) <= TOL_F64


def test_update_enqueued_ahead_of_status_with_wrong_hints(E):
    """With a degree hint the update is enqueued right after each status
    read-back and runs only once the loop has stopped.  Steps whose hint is
    too small (several batches) or too large (guarded launches past the
    stop) still give the oracle's result, for Euler steps and for phi_1 with
    several substeps."""
    shape = (256, 10, 7)
    op, A = make(E, shape, "neumann0", "separable")
    n = int(np.prod(shape))
    a, b = O.gershgorin_interval(A)
    smooth = 0.5 + 1e-6 * synth.uniform_vector(n, 4)
    rough = 0.5 + 0.4 * synth.uniform_vector(n, 5)
    tau = 20.0 / (b - a)
    for name, u0 in (("smooth", smooth), ("rough", rough), ("smooth", smooth), ("rough", rough)):
        u = T(u0)
        print(f"euler with hint: {name}", flush=True)
        st = E.expeuler_step(op, tau, u, tol=1e-10)
        uo, so = I.expeuler_step(A, tau, u0, 1e-10)
        assert relerr(N(u), uo) <= TOL_F64, (name, relerr(N(u), uo))
        assert abs(st["degree_last"] - so.degrees[-1]) <= 1
    tau3 = 230.0 / (b - a)                      # three substeps
    for name, v in (("smooth", smooth), ("rough", rough), ("smooth", smooth)):
        print(f"phi1 with hint: {name}", flush=True)
        y, st = E.phi_action(op, 1, tau3, T(v), tol=1e-10)
        yo, so = I.phi_action(A, 1, tau3, v, 1e-10)
        assert st["substeps"] == 3
        assert relerr(N(y), yo) <= TOL_F64, (name, relerr(N(y), yo))


def test_pair_fp32_rows_of_512(E):
    """FP32 storage on rows of 512 points (four waves per row, two output
    rows per workgroup): pair sweeps are taken and agree with the oracle
    to the FP32 bar."""
    shape = (512, 6, 8)
    op, A = make(E, shape, "neumann0", "separable")
    v = synth.uniform_vector(int(np.prod(shape)), 9)
    a, b = O.gershgorin_interval(A)
    tau = 10.0 / (b - a)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10, dtype="f32", params=E.LejaParams(profile=True))
    yo, _ = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(y), yo) <= 5e-6
    assert st["timed_pairs"] >= 1


def test_fused_start_fp32_rows_of_512(E):
    """The FP32 fused start on rows of 512 points (four waves per row, the
    FP64 w_j ring at its largest), against the separate start and the
    oracle."""
    shape = (512, 6, 8)
    op, A = make(E, shape, "neumann0", "separable")
    n = int(np.prod(shape))
    u0 = 0.5 + 0.1 * synth.uniform_vector(n, 14)
    a, b = O.gershgorin_interval(A)
    tau = 15.0 / (b - a)
    uo, _ = I.expeuler_step(A, tau, u0, 1e-10)
    got = {}
    for fs in (1, 2):
        u = T(u0)
        st = E.expeuler_step(op, tau, u, tol=1e-10, dtype="f32", params=E.LejaParams(fuse_start=fs))
        assert st["fused_starts"] == (1 if fs == 2 else 0)
        assert relerr(N(u), uo) <= 5e-6
        got[fs] = N(u)
    assert relerr(got[2], got[1]) <= 1e-5
