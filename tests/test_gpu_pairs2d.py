"""GPU parity of the 2D pair sweep (two Newton products per pass on 2D
constant-coefficient stencils).

phi_1(tau A) v on 2D grids with the pair sweep on (the default where it
applies) against the FP64 oracle and against the single-product path on
the same inputs: the 128 x 128 Dirichlet Laplacian of the plain-method
workload, strips ragged against the 64- and 128-point tile width, odd row
lengths (one point per lane), single rows and columns, the three boundary
handlings, FP32 storage, and stops after either product of a pair.
"""
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


def make(E, shape, bc, coef=1.3):
    h = tuple(1.0 / (s + 1) for s in shape)
    return E.StencilOp(shape, h, bc, coef=coef), O.stencil_matrix(shape, h, bc, coef=coef)


def run_pair_and_single(E, op, v, tau, tol, dtype="f64", interval=None):
    yp, sp = E.phi_action(op, 1, tau, T(v), tol=tol, dtype=dtype,
                          params=E.LejaParams(profile=True, interval=interval))
    ys, ss = E.phi_action(op, 1, tau, T(v), tol=tol, dtype=dtype,
                          params=E.LejaParams(pairs=False, profile=True, interval=interval))
    return N(yp), sp, N(ys), ss


SHAPES = [
    (128, 128),   # the plain-method grid: one 128-point strip per row
    (130, 37),    # two strips, the second 2 points wide; rows ragged against the tile
    (129, 33),    # odd rows: one point per lane, three strips
    (64, 1),      # a single row
    (1, 50),      # a single column
    (2, 3),       # tiny
    (300, 17),    # ragged third strip
    (1000, 9),    # eight strips
    (257, 70),    # odd, five 64-point strips, several row tiles
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["dirichlet0", "neumann0", "interior_only"])
def test_pair2d_phi1_matches_oracle(E, shape, bc):
    op, A = make(E, shape, bc)
    n = int(np.prod(shape))
    v = synth.uniform_vector(n, 11)
    a, b = O.gershgorin_interval(A)
    # interior_only with a side of at most 2 points has no interior: A = 0
    # and a = b, so both sides get the interval [-1, 0] instead
    iv = None if b > a else (-1.0, 0.0)
    tau = 8.0 / (b - a) if iv is None else 1e-3   # tau (b - a) = 8: one substep of a few dozen products
    print(f"pair2d phi1 {shape} {bc}", flush=True)
    yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-10, interval=iv)
    yo, so = I.phi_action(A, 1, tau, v, 1e-10, interval=iv)
    assert relerr(yp, yo) <= TOL_F64, relerr(yp, yo)
    assert relerr(ys, yo) <= TOL_F64
    assert abs(sp["degree_last"] - so.degrees[-1]) <= 1
    # the pair path took pair sweeps; the pair over products 0 and 1 is not
    # timed, so a stop at m = 2 shows none
    assert sp["degree_last"] <= 2 or sp["timed_pairs"] >= 1
    assert ss["timed_pairs"] == 0


def test_pair2d_plain_workload(E):
    """The plain-method case: 128 x 128 Dirichlet Laplacian, h = 1/129,
    tau = 1e-4, tolerance 1e-10, several substeps."""
    shape = (128, 128)
    op, A = make(E, shape, "dirichlet0", coef=1.0)
    v = synth.uniform_vector(128 * 128, 0)
    print("pair2d plain workload", flush=True)
    yp, sp, ys, ss = run_pair_and_single(E, op, v, 1e-4, 1e-10)
    yo, so = I.phi_action(A, 1, 1e-4, v, 1e-10)
    assert relerr(yp, yo) <= TOL_F64
    assert relerr(ys, yo) <= TOL_F64
    assert sp["timed_pairs"] >= 1


@pytest.mark.parametrize("shape", [(128, 128), (129, 33), (300, 17), (130, 37), (1000, 9), (4, 7)])
def test_pair2d_f32_storage(E, shape):
    """FP32 storage: pairs and singles both within the FP32 error of the
    FP64 oracle (four points per lane where rows have a multiple of 4
    points, else two or one)."""
    op, A = make(E, shape, "neumann0")
    n = int(np.prod(shape))
    v = synth.uniform_vector(n, 5)
    a, b = O.gershgorin_interval(A)
    tau = 8.0 / (b - a)
    print(f"pair2d f32 {shape}", flush=True)
    yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-6, dtype="f32")
    yo, _ = I.phi_action(A, 1, tau, v, 1e-12)
    assert relerr(yp, yo) <= 2e-5, relerr(yp, yo)
    assert relerr(ys, yo) <= 2e-5
    assert sp["timed_pairs"] >= 1


def test_pair2d_stops_after_either_product(E):
    """Vary tau so the stop falls after the first and after the second
    product of a pair; both match the oracle, the first with the extra term
    removed."""
    shape = (200, 23)
    op, A = make(E, shape, "dirichlet0")
    v = synth.uniform_vector(200 * 23, 3)
    a, b = O.gershgorin_interval(A)
    parities = set()
    for q in np.linspace(2.0, 40.0, 12):
        tau = q / (b - a)
        print(f"pair2d stop q={q:.2f}", flush=True)
        yp, sp, ys, ss = run_pair_and_single(E, op, v, tau, 1e-10)
        yo, so = I.phi_action(A, 1, tau, v, 1e-10)
        assert relerr(yp, yo) <= TOL_F64, (q, relerr(yp, yo))
        assert sp["degree_last"] == ss["degree_last"]
        parities.add(sp["degree_last"] % 2)
    assert parities == {0, 1}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("rows", [4, 8, 16, 32, 64])
def test_pair2d_every_tile_height(E, rows, dtype):
    """The operator's pair setting fixes the tile height: every allowed
    height gives the oracle's result (tiles ragged against the grid's rows
    and taller than it; one, two and, in FP32, four points per lane)."""
    tol, bound = (1e-10, TOL_F64) if dtype == "f64" else (1e-6, 2e-5)
    for shape, bc in (((300, 70), "dirichlet0"), ((129, 33), "neumann0"), ((64, 5), "dirichlet0"),
                      ((258, 9), "neumann0"), ((132, 21), "interior_only")):
        op, A = make(E, shape, bc)
        op.set_pairs(rows)
        assert op.pair_setting() == rows
        n = int(np.prod(shape))
        v = synth.uniform_vector(n, 21)
        a, b = O.gershgorin_interval(A)
        tau = 8.0 / (b - a)
        print(f"pair2d rows={rows} {dtype} {shape} {bc}", flush=True)
        yp, sp = E.phi_action(op, 1, tau, T(v), tol=tol, dtype=dtype, params=E.LejaParams(profile=True))
        yo, _ = I.phi_action(A, 1, tau, v, 1e-12)
        assert relerr(N(yp), yo) <= bound, relerr(N(yp), yo)
        assert sp["timed_pairs"] >= 1


def test_pair2d_autotuned_height(E, tmp_path):
    """The autotuner times the 2D pair sweep at several tile heights, keeps
    the fastest (or single products), a fresh operator takes the cached
    choice, and the result still matches the oracle."""
    from paper_1309_4616_amd import autotune
    cache = str(tmp_path / "tiles.json")
    shape = (512, 300)
    op, A = make(E, shape, "dirichlet0")
    print("pair2d autotune", flush=True)
    res = autotune.tune(op, "f64", reps=3, path=cache)
    heights = sorted(c[1] for c, _ in res["candidates"] if c[0] == 0)
    assert heights == [4, 8, 16, 32, 64]
    setting = op.pair_setting()
    assert setting in (0, 4, 8, 16, 32, 64)
    if setting:
        best = min((t, c[1]) for c, t in res["candidates"] if c[0] == 0)[1]
        assert setting == best and res["pair_rows"] == best
    op2, _ = make(E, shape, "dirichlet0")
    assert autotune.load(op2, "f64", path=cache)
    assert op2.pair_setting() == setting and op2.tiles() == op.tiles()
    v = synth.uniform_vector(512 * 300, 4)
    a, b = O.gershgorin_interval(A)
    tau = 8.0 / (b - a)
    yp, _ = E.phi_action(op, 1, tau, T(v), tol=1e-10)
    yo, _ = I.phi_action(A, 1, tau, v, 1e-10)
    assert relerr(N(yp), yo) <= TOL_F64
