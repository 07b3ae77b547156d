"""GPU parity: the HIP library against the FP64 oracle on seeded inputs.

Every test calls the C ABI through the Python binding and compares with
``oracle`` element by element (relative 2-norm, FP64 bar 1e-10), at sizes
that span several tiles and leave ragged tails; full sizes are checked on
sampled points and through invariants that hold at any size.
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


def stencil_pair(E, shape, h, bc, coef_kind, seed=0):
    """(GPU op, oracle matrix) for the same operator."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    if coef_kind == "const":
        return E.StencilOp(shape, h, bc, coef=1.7), O.stencil_matrix(shape, h, bc, coef=1.7)
    if coef_kind == "separable":
        tabs = [np.sin(2 * math.pi * (np.arange(s) + 0.5) / s) for s in shape]
        c0, c1 = 1.0, 0.6
        prod = tabs[0][None, :]
        if len(shape) == 2:
            fld = c0 + c1 * (tabs[1][:, None] * tabs[0][None, :])
        else:
            fld = c0 + c1 * ((tabs[2][:, None, None] * tabs[1][None, :, None]) * tabs[0][None, None, :])
        del prod
        op = E.StencilOp(shape, h, bc, coef=("separable", c0, c1, *tabs))
        return op, O.stencil_matrix(shape, h, bc, coef=fld.reshape(-1))
    fld = 1.0 + rng.uniform(0, 1, size=n)
    return E.StencilOp(shape, h, bc, coef=fld), O.stencil_matrix(shape, h, bc, coef=fld)


# ---------------------------------------------------------------------------
# the small 2D workload: 128^2 interior, Dirichlet, tau = 1e-4, tol 1e-10
# ---------------------------------------------------------------------------

def test_phi1_2d_dirichlet_128(E):
    Nn = 128
    h = 1.0 / (Nn + 1)
    v = synth.uniform_vector(Nn * Nn, 0)
    op = E.StencilOp((Nn, Nn), (h, h), "dirichlet0")
    y, st = E.phi_action(op, 1, 1e-4, T(v), tol=1e-10)
    A = O.stencil_matrix((Nn, Nn), (h, h), "dirichlet0")
    yo, sto = I.phi_action(A, 1, 1e-4, v, 1e-10)
    assert relerr(N(y), yo) <= TOL_F64
    assert st["converged"] == 1 and st["substeps"] == 1
    assert abs(st["degree_last"] - sto.degrees[0]) <= 1
    assert st["interval_a"] == pytest.approx(-133128.0, rel=1e-14)
    assert abs(st["interval_b"]) <= 1e-9
    # and against the DST closed form
    j = np.arange(1, Nn + 1)
    s2 = np.sin(j * math.pi * h / 2) ** 2
    z = 1e-4 * (-(4 / h ** 2) * (s2[:, None] + s2[None, :]))
    import scipy.fft as F
    V = v.reshape(Nn, Nn)
    exact = F.dstn(np.expm1(z) / z * F.dstn(V, type=1, norm="ortho"), type=1, norm="ortho").reshape(-1)
    assert relerr(N(y), exact) <= TOL_F64


# ---------------------------------------------------------------------------
# the product of eq. (3)
# ---------------------------------------------------------------------------

SHAPES = [(100, 37), (64, 33), (1, 9), (70, 33, 21), (64, 4, 17), (3, 1, 7), (130, 5, 40)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
@pytest.mark.parametrize("coef", ["const", "separable", "field"])
def test_apply_op_matches_oracle(E, shape, bc, coef):
    h = tuple(1.0 / (s + 1) for s in shape)
    op, A = stencil_pair(E, shape, h, bc, coef, seed=len(shape))
    x = synth.uniform_vector(int(np.prod(shape)), 3)
    y = E.apply_op(op, 0.37, -1.25, T(x))
    want = O.apply_op(A, 0.37, -1.25, x)
    scale = max(np.abs(want).max(), 1.0)
    assert np.max(np.abs(N(y) - want)) <= 1e-13 * scale


@pytest.mark.parametrize("shape", [(100, 37), (70, 33, 21)])
def test_apply_op_fp32(E, shape):
    import torch
    h = tuple(1.0 / (s + 1) for s in shape)
    op, A = stencil_pair(E, shape, h, "neumann0", "separable")
    x = synth.uniform_vector(int(np.prod(shape)), 4)
    y = E.apply_op(op, 1.0 / abs(O.gershgorin_interval(A)[0]), 0.5, T(x).to(torch.float32))
    want = O.apply_op(A, 1.0 / abs(O.gershgorin_interval(A)[0]), 0.5, x)
    assert relerr(N(y).astype(np.float64), want) <= 1e-6


@pytest.mark.parametrize("shape,bc,coef", [((100, 37), "dirichlet0", "const"),
                                           ((70, 33, 21), "neumann0", "separable"),
                                           ((40, 22, 17), "dirichlet0", "field"),
                                           ((20, 20, 20), "interior_only", "const")])
def test_interval_matches_oracle(E, shape, bc, coef):
    h = tuple(1.0 / (s + 1) for s in shape)
    op, A = stencil_pair(E, shape, h, bc, coef)
    a, b = op.interval()
    ao, bo = O.gershgorin_interval(A)
    assert a == pytest.approx(ao, rel=1e-13)
    assert abs(b - bo) <= 1e-12 * abs(ao)


# ---------------------------------------------------------------------------
# phi_k on 3D variable-coefficient operators, substeps, k = 0 and 2
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("coef", ["separable", "field"])
def test_phi1_3d_variable_neumann(E, coef):
    shape = (67, 45, 37)
    h = (1 / 67, 1 / 45, 1 / 37)
    op, A = stencil_pair(E, shape, h, "neumann0", coef, seed=5)
    a, b = O.gershgorin_interval(A)
    tau = 40.0 / (b - a)
    v = synth.uniform_vector(A.shape[0], 6)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10)
    yo, sto = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(y), yo) <= TOL_F64
    # mass: 1^T phi_1(tau A) v = 1^T v under zero-flux boundaries
    assert abs(N(y).sum() - v.sum()) <= 1e-9 * np.abs(v).sum()


@pytest.mark.parametrize("k,tau,shape", [(1, 2e-2, (40, 40)), (0, 2e-2, (40, 40)),
                                         (2, 1e-3, (50, 31)), (0, 1e-4, (50, 31)),
                                         (1, 3e-3, (30, 26, 19))])
def test_phi_k_and_substeps(E, k, tau, shape):
    h = tuple(1.0 / (s + 1) for s in shape)
    op, A = stencil_pair(E, shape, h, "dirichlet0", "const")
    v = synth.uniform_vector(A.shape[0], 8)
    y, st = E.phi_action(op, k, tau, T(v), tol=1e-10)
    yo, sto = I.phi_action(A, k, tau, v, 1e-10)
    assert st["substeps"] == sto.substeps
    assert relerr(N(y), yo) <= TOL_F64


def test_supplied_interval_and_limits(E):
    shape = (50, 40)
    h = (0.02, 0.025)
    op, A = stencil_pair(E, shape, h, "neumann0", "const")
    a, b = O.gershgorin_interval(A)
    iv = (1.3 * a, 0.0)
    v = synth.uniform_vector(A.shape[0], 9)
    params = E.LejaParams(l_max=30.0, m_max=60, interval=iv)
    y, st = E.phi_action(op, 1, 80.0 / (b - a), T(v), tol=1e-10, params=params)
    yo, sto = I.phi_action(A, 1, 80.0 / (b - a), v, 1e-10, interval=iv,
                           params=I.LejaParams(l_max=30.0, m_max=60))
    assert st["substeps"] == sto.substeps >= 3
    assert relerr(N(y), yo) <= TOL_F64


def test_nonconvergence_retries_then_converges(E):
    shape = (20, 20)
    h = (1 / 21, 1 / 21)
    op, A = stencil_pair(E, shape, h, "dirichlet0", "const")
    v = synth.uniform_vector(400, 1)
    tau = 60.0 / (8.0 / h[0] ** 2 * 1.7)
    p = dict(l_max=1000.0, m_max=20, max_retries=4)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10, params=E.LejaParams(**p))
    yo, sto = I.phi_action(A, 1, tau, v, 1e-10, params=I.LejaParams(**p))
    assert st["retries"] == sto.retries >= 1
    assert relerr(N(y), yo) <= TOL_F64


def test_error_paths(E):
    import torch
    shape = (20, 20)
    h = (1 / 21, 1 / 21)
    op = E.StencilOp(shape, h, "dirichlet0")
    v = T(synth.uniform_vector(400, 1))
    with pytest.raises(E.ExpiError) as ei:
        E.phi_action(op, 1, 1.0, v, tol=1e-10, params=E.LejaParams(l_max=1e6, m_max=5, max_retries=0))
    assert ei.value.name == "ENOTCONV"
    bad = v.clone()
    bad[17] = float("nan")
    with pytest.raises(E.ExpiError) as ei:
        E.phi_action(op, 1, 1e-3, bad, tol=1e-10)
    assert ei.value.name == "ENONFINITE"
    u = v.clone()
    u[3] = float("inf")
    u_before = u.clone()
    with pytest.raises(E.ExpiError) as ei:
        E.expeuler_step(op, 1e-3, u, tol=1e-10)
    assert ei.value.name == "ENONFINITE"
    assert torch.equal(u, u_before)          # left unchanged on error
    # zero vector and tau = 0
    y, st = E.phi_action(op, 1, 1e-3, torch.zeros_like(v), tol=1e-10)
    assert torch.count_nonzero(y).item() == 0
    y, st = E.phi_action(op, 1, 0.0, v, tol=1e-10)
    assert torch.allclose(y, v, rtol=1e-15, atol=0)


def test_deterministic(E):
    shape = (70, 33, 21)
    h = tuple(1.0 / s for s in shape)
    op, A = stencil_pair(E, shape, h, "neumann0", "separable")
    v = T(synth.uniform_vector(A.shape[0], 2))
    y1, s1 = E.phi_action(op, 1, 3e-3, v, tol=1e-10)
    y2, s2 = E.phi_action(op, 1, 3e-3, v, tol=1e-10)
    assert s1["degree_last"] == s2["degree_last"]
    assert s1["err_est"] == s2["err_est"]
    assert np.array_equal(N(y1), N(y2))


# ---------------------------------------------------------------------------
# exponential Euler: the 3D reaction-diffusion problem
# ---------------------------------------------------------------------------

def rd_problem(E, n, amp=0.5):
    h = 1.0 / n
    coef = synth.sine_coefficient(n, amp)
    op = E.StencilOp((n, n, n), (h, h, h), "neumann0",
                     coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))
    return op, coef


def test_expeuler_3d_reaction_diffusion_64(E):
    n = 64
    op, coef = rd_problem(E, n)
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=coef.field())
    a, b = O.gershgorin_interval(A)
    tau = 1e-5 * (256 / n) ** 2   # same stiffness tau*(b-a) as the 256^3 grid at 1e-5
    u0 = synth.gaussian_bump_3d(n, seed=0)
    u = T(u0)
    uo = u0.copy()
    for step in range(3):
        mass_before = N(u).sum()
        g = N(u) - N(u) ** 3
        st = E.expeuler_step(op, tau, u, tol=1e-10)
        uo, sto = I.expeuler_step(A, tau, uo, 1e-10, interval=(a, b))
        assert relerr(N(u), uo) <= TOL_F64, step
        assert st["interval_a"] == pytest.approx(a, rel=1e-13)
        # mass identity under zero-flux boundaries
        assert abs(N(u).sum() - (mass_before + tau * g.sum())) <= 1e-9 * np.abs(N(u)).sum()


def test_expeuler_substeps(E):
    n = 24
    op, coef = rd_problem(E, n, amp=0.7)
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=coef.field())
    a, b = O.gershgorin_interval(A)
    tau = 350.0 / (b - a)
    u0 = 0.5 * synth.gaussian_bump_3d(n, seed=2)
    u = T(u0)
    st = E.expeuler_step(op, tau, u, tol=1e-10)
    uo, sto = I.expeuler_step(A, tau, u0, 1e-10)
    assert st["substeps"] == sto.substeps >= 4
    assert relerr(N(u), uo) <= TOL_F64


def test_expeuler_fp32_storage(E):
    n = 48
    op, coef = rd_problem(E, n)
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=coef.field())
    tau = 1e-5 * (256 / n) ** 2
    u0 = synth.gaussian_bump_3d(n, seed=1)
    u = T(u0)
    st = E.expeuler_step(op, tau, u, tol=1e-8, dtype="f32")
    uo, _ = I.expeuler_step(A, tau, u0, 1e-12)
    # FP32 storage of the Newton vectors: the increment u1 - u0 carries the
    # FP32 rounding; the full state is much more accurate
    err_inc = relerr(N(u) - u0, uo - u0)
    assert err_inc <= 5e-5, err_inc
    assert relerr(N(u), uo) <= 1e-6


def test_phi1_fp32_storage_2d(E):
    Nn = 128
    h = 1.0 / (Nn + 1)
    v = synth.uniform_vector(Nn * Nn, 0)
    op = E.StencilOp((Nn, Nn), (h, h), "dirichlet0")
    y, st = E.phi_action(op, 1, 1e-4, T(v), tol=1e-8, dtype="f32")
    yo, _ = I.phi_action(O.stencil_matrix((Nn, Nn), (h, h), "dirichlet0"), 1, 1e-4, v, 1e-12)
    assert relerr(N(y), yo) <= 5e-6


# ---------------------------------------------------------------------------
# CSR: negative graph Laplacian of a random geometric graph
# ---------------------------------------------------------------------------

def csr_pair(E, n, seed, mean_degree=26.0):
    g = synth.rgg_negative_laplacian(n, seed=seed, mean_degree=mean_degree)
    op = E.CsrOp(g.n, g.rowptr, g.colind, g.val)
    return op, O.csr_matrix(g.n, g.rowptr, g.colind, g.val), g


def test_csr_apply_and_interval(E):
    op, A, g = csr_pair(E, 20011, seed=3)
    x = synth.uniform_vector(g.n, 4)
    y = E.apply_op(op, -0.5, 2.0, T(x))
    want = O.apply_op(A, -0.5, 2.0, x)
    assert np.max(np.abs(N(y) - want)) <= 1e-13 * np.abs(want).max()
    a, b = op.interval()
    ao, bo = O.gershgorin_interval(A)
    assert a == ao and b == bo


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_csr_uneven_rows_apply(E, lanes):
    """Rows of 0, 1..40 and 300 stored entries (duplicate columns allowed):
    empty rows, waves whose entries run past the LDS stage into the direct
    tail, and a ragged last row block, for each lane count."""
    rng = np.random.default_rng(11)
    n = 5003
    deg = rng.integers(1, 41, size=n)
    deg[::97] = 0
    deg[5::101] = 300
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    nnz = int(rowptr[-1])
    colind = rng.integers(0, n, size=nnz).astype(np.int32)
    val = rng.standard_normal(nnz)
    op = E.CsrOp(n, rowptr, colind, val)
    op.set_tiles(lanes, 4, 1)
    A = O.csr_matrix(n, rowptr, colind, val)
    x = synth.uniform_vector(n, 7)
    y = E.apply_op(op, 0.75, -1.5, T(x))
    want = O.apply_op(A, 0.75, -1.5, x)
    assert np.max(np.abs(N(y) - want)) <= 1e-13 * np.abs(want).max()


def test_csr_phi1(E):
    op, A, g = csr_pair(E, 30007, seed=5)
    rho = synth.spectral_radius_symmetric(g)
    tau = 50.0 / rho
    v = synth.uniform_vector(g.n, 6)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10)
    yo, sto = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(y), yo) <= TOL_F64
    assert abs(N(y).sum() - v.sum()) <= 1e-9 * np.abs(v).sum()


@pytest.mark.slow
def test_csr_phi1_full_size(E):
    """n = 2^20 rows, ~27 stored entries per row, tau rho(A) = 50, tol 1e-10."""
    op, A, g = csr_pair(E, 1 << 20, seed=0)
    rho = synth.spectral_radius_symmetric(g)
    tau = 50.0 / rho
    v = synth.uniform_vector(g.n, 0)
    y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10)
    yo, sto = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(y), yo) <= TOL_F64
    assert 20 <= g.nnz / g.n <= 30


# ---------------------------------------------------------------------------
# full-size 3D grid: sampled points and invariants
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_full_size_256_apply_samples_and_step_invariants(E):
    import torch
    n = 256
    op, coef = rd_problem(E, n)
    h = 1.0 / n
    u0 = synth.gaussian_bump_3d(n, seed=0)
    u = T(u0)
    # the product at sampled points (boundary faces, edges, corners and interior)
    y = E.apply_op(op, 1.0, 0.0, u)
    rng = np.random.default_rng(0)
    pts = np.concatenate([rng.choice(n ** 3, size=400, replace=False),
                          [0, n - 1, n * n - 1, n ** 3 - 1, n * n * (n - 1), 5 * n * n + 7]])
    want = O.apply_at((n, n, n), (h, h, h), "neumann0", u0, pts, coef=coef.field())
    got = N(y)[pts]
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()
    # one exponential Euler step at tol 1e-8: mass identity, and the step
    # equals u + tau * phi_1(tau A) F(u) evaluated separately
    g = u0 - u0 ** 3
    st = E.expeuler_step(op, 1e-5, u, tol=1e-10)
    assert st["substeps"] == 1 and st["converged"] == 1
    assert abs(N(u).sum() - (u0.sum() + 1e-5 * g.sum())) <= 1e-9 * np.abs(u0).sum()
    F = E.apply_op(op, 1.0, 0.0, T(u0)) + T(g)
    pf, _ = E.phi_action(op, 1, 1e-5, F, tol=1e-10)
    assert relerr(N(u), u0 + 1e-5 * N(pf)) <= 1e-12
    del F, pf
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# autotuner: candidate timings, cached choice, unchanged results
# ---------------------------------------------------------------------------

def test_autotune_stencil_and_csr(E, tmp_path):
    cache = str(tmp_path / "tiles.json")
    shape = (96, 64, 48)
    h = tuple(1.0 / s for s in shape)
    op, A = stencil_pair(E, shape, h, "neumann0", "separable")
    v = synth.uniform_vector(A.shape[0], 3)
    y0, _ = E.phi_action(op, 1, 2e-3, T(v), tol=1e-10)
    entry = E.autotune.tune(op, "f64", reps=3, path=cache)
    # 32 single-product settings, then the pair sweep (0, 0, 2)
    assert len(entry["candidates"]) == 33
    singles = [t for c, t in entry["candidates"] if c[0] != 0]
    pair_us = [t for c, t in entry["candidates"] if c == [0, 0, 2]]
    assert len(singles) == 32 and len(pair_us) == 1
    assert tuple(entry["tiles"]) == op.tiles()
    assert entry["us"] == min(singles)
    assert entry["pairs"] == (0.5 * pair_us[0] < min(singles)) == op.pairs()
    y1, _ = E.phi_action(op, 1, 2e-3, T(v), tol=1e-10)
    assert relerr(N(y1), N(y0)) <= 1e-12
    yo, _ = I.phi_action(A, 1, 2e-3, v, 1e-10)
    assert relerr(N(y1), yo) <= TOL_F64
    # a fresh operator picks the cached setting without timing
    op2, _ = stencil_pair(E, shape, h, "neumann0", "separable")
    op2.set_pairs(not op.pairs())
    assert E.autotune.load(op2, "f64", path=cache)
    assert op2.tiles() == op.tiles() and op2.pairs() == op.pairs()
    # single products on request, the same result to rounding
    op2.set_pairs(False)
    y2, st2 = E.phi_action(op2, 1, 2e-3, T(v), tol=1e-10, params=E.LejaParams(profile=True))
    assert st2["timed_pairs"] == 0
    assert relerr(N(y2), N(y0)) <= 1e-12
    # CSR lanes per row
    cop, CA, g = csr_pair(E, 20011, seed=3)
    centry = E.autotune.tune(cop, "f64", reps=3, path=cache)
    assert len(centry["candidates"]) == 12 and centry["pairs"] is None
    x = synth.uniform_vector(g.n, 4)
    y = E.apply_op(cop, -0.5, 2.0, T(x))
    assert np.max(np.abs(N(y) - O.apply_op(CA, -0.5, 2.0, x))) <= 1e-13 * np.abs(N(y)).max()


# ---------------------------------------------------------------------------
# many uneven 2D problems in one persistent launch
# ---------------------------------------------------------------------------

def batch_case(seed=0, count=12):
    rng = np.random.default_rng(seed)
    nx = rng.integers(9, 90, size=count)
    ny = rng.integers(9, 90, size=count)
    nx[0], ny[0] = 64, 64
    nx[1], ny[1] = 1, 30          # degenerate row
    hx, hy = 1.0 / (nx + 1.0), 1.0 / (ny + 1.0)
    tau = 10 ** rng.uniform(-5, -2.3, size=count)
    return nx, ny, hx, hy, tau


def batch_oracle(nx, ny, hx, hy, tau, v_all, off, bc, tol):
    out = []
    for i in range(len(nx)):
        n = int(nx[i] * ny[i])
        A = O.stencil_matrix((int(nx[i]), int(ny[i])), (hx[i], hy[i]), bc)
        a = -4.0 * (1 / hx[i] ** 2 + 1 / hy[i] ** 2)
        y, st = I.phi_action(A, 1, tau[i], v_all[off[i]:off[i] + n], tol, interval=(a, 0.0))
        out.append((y, st))
    return out


@pytest.mark.parametrize("dtype,bc", [("f64", "dirichlet0"), ("f32", "dirichlet0"), ("f64", "neumann0")])
def test_batch_matches_oracle_per_instance(E, dtype, bc):
    import torch
    nx, ny, hx, hy, tau = batch_case()
    b = E.Batch(nx, ny, hx, hy, tau, bc=bc, tol=1e-10, dtype=dtype)
    v_all = synth.uniform_vector(b.total_length, 11)
    v = T(v_all)
    y = torch.zeros_like(v)
    b.prepare()
    b.launch_persistent(v, y)
    stats, rounds = b.results()
    want = batch_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, bc, 1e-10)
    yy = N(y)
    bar = TOL_F64 if dtype == "f64" else 5e-6
    for i, (yo, sto) in enumerate(want):
        n = int(nx[i] * ny[i])
        got = yy[b.offsets[i]:b.offsets[i] + n]
        assert relerr(got, yo) <= bar, (i, relerr(got, yo))
        assert stats[i]["status"] == 0 and stats[i]["substeps"] == sto.substeps
        if dtype == "f64":
            assert abs(stats[i]["degree_last"] - sto.degrees[-1]) <= 1
    # a round takes at most two products per instance
    assert rounds >= max((s["newton_steps"] + 1) // 2 for s in stats)


def test_batch_graph_replays_are_identical(E):
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=3, count=20)
    b = E.Batch(nx, ny, hx, hy, tau, tol=1e-8, dtype="f32")
    v = T(synth.uniform_vector(b.total_length, 5))
    y_eager = torch.zeros_like(v)
    b.prepare()
    b.launch_persistent(v, y_eager)
    s_eager, r_eager = b.results()
    y = torch.zeros_like(v)
    b.capture_persistent(v, y)
    mask = torch.zeros(b.total_length, dtype=torch.bool, device=v.device)
    for i in range(b.count):
        mask[int(b.offsets[i]):int(b.offsets[i]) + int(nx[i] * ny[i])] = True
    for rep in range(3):
        y.fill_(float("nan"))
        b.replay()
        torch.cuda.synchronize()
        s_rep, r_rep = b.results()
        assert r_rep == r_eager
        assert torch.equal(y[mask], y_eager[mask]), rep
        assert [s["newton_steps"] for s in s_rep] == [s["newton_steps"] for s in s_eager]


@pytest.mark.parametrize("pairs", [True, False])
def test_batch_persistent_equals_rounds(E, pairs):
    """The persistent launch and the eager rounds run the same tiles and
    combine each instance's partials in the same order (two Newton products
    per round, and one)."""
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=5, count=24)
    b = E.Batch(nx, ny, hx, hy, tau, tol=1e-9, dtype="f64")
    b.set_pairs(pairs)
    v = T(synth.uniform_vector(b.total_length, 8))
    y0 = torch.zeros_like(v)
    y1 = torch.zeros_like(v)
    b.prepare()
    b.launch(v, y0)
    s0, r0 = b.results()
    b.launch_persistent(v, y1)
    s1, r1 = b.results()
    assert r1 == r0
    assert [s["newton_steps"] for s in s1] == [s["newton_steps"] for s in s0]
    mask = torch.zeros(b.total_length, dtype=torch.bool, device=v.device)
    for i in range(b.count):
        mask[int(b.offsets[i]):int(b.offsets[i]) + int(nx[i] * ny[i])] = True
    assert torch.equal(y1[mask], y0[mask])
