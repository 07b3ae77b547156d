"""GPU parity of the batched solver (many uneven 2D problems, run in rounds).

Each instance is compared with the oracle on its own: the Leja oracle
(phi_action on the assembled matrix, same interval) at small sizes, the
sine-mode closed form at larger ones.  The solver forms two Newton products
per round by default; one per round is compared too.  The captured graph is replayed with
eager work in between and every replay is compared with the eager run.
"""
import numpy as np
import pytest

import synth
from oracle import integrators as I
from oracle import operators as O

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10
TOL_F32 = 5e-6


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


def batch_case(seed=0, count=12):
    """Uneven sizes with ragged tails, a one-column instance and a 64^2 one."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(9, 90, size=count)
    ny = rng.integers(9, 90, size=count)
    nx[0], ny[0] = 64, 64
    nx[1], ny[1] = 1, 30
    hx, hy = 1.0 / (nx + 1.0), 1.0 / (ny + 1.0)
    tau = 10 ** rng.uniform(-5, -2.3, size=count)
    return nx, ny, hx, hy, tau


def leja_oracle(nx, ny, hx, hy, tau, v_all, off, bc, tol, coef=1.0):
    out = []
    for i in range(len(nx)):
        n = int(nx[i] * ny[i])
        A = O.stencil_matrix((int(nx[i]), int(ny[i])), (hx[i], hy[i]), bc, coef=coef)
        a = -4.0 * coef * (1 / hx[i] ** 2 + 1 / hy[i] ** 2)
        y, st = I.phi_action(A, 1, tau[i], v_all[off[i]:off[i] + n], tol, interval=(a, 0.0))
        out.append((y, st))
    return out


def run(E, nx, ny, hx, hy, tau, seed=11, **kw):
    import torch
    b = E.Batch(nx, ny, hx, hy, tau, **kw)
    v_all = synth.uniform_vector(b.total_length, seed)
    v = T(v_all)
    y = torch.zeros_like(v)
    b.prepare()
    print(f"batch launch: count={b.count} kw={kw}", flush=True)
    b.launch(v, y)
    stats, rounds = b.results()
    return b, v_all, N(y), stats, rounds


@pytest.mark.parametrize("dtype,bc", [("f64", "dirichlet0"), ("f32", "dirichlet0"), ("f64", "neumann0"),
                                      ("f32", "neumann0")])
def test_batch_matches_leja_oracle_per_instance(E, dtype, bc):
    nx, ny, hx, hy, tau = batch_case()
    b, v_all, yy, stats, rounds = run(E, nx, ny, hx, hy, tau, bc=bc, tol=1e-10, dtype=dtype)
    want = leja_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, bc, 1e-10)
    bar = TOL_F64 if dtype == "f64" else TOL_F32
    for i, (yo, sto) in enumerate(want):
        n = int(nx[i] * ny[i])
        got = yy[b.offsets[i]:b.offsets[i] + n]
        assert relerr(got, yo) <= bar, (i, relerr(got, yo))
        assert stats[i]["status"] == 0 and stats[i]["substeps"] == sto.substeps
        if dtype == "f64":
            # the stop test sees the same norms up to summation order; a pair
            # of products that stops after its first one has formed one more
            assert abs(stats[i]["degree_last"] - sto.degrees[-1]) <= 1
            assert -sto.substeps <= stats[i]["newton_steps"] - sum(sto.degrees) <= 2 * sto.substeps
    # each round advances every unfinished instance by one step of at most
    # two products
    assert b.pairs
    longest = max(s["newton_steps"] + 2 * s["substeps"] for s in stats)
    assert max((s["newton_steps"] + 1) // 2 for s in stats) <= rounds <= min(longest, b.max_rounds)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_pairs_against_single_products(E, dtype):
    """Two products per round against one per round on the same batch: the
    same degrees up to one (the stop test sees the same norms up to the
    order of the sums), products formed at most one more per substep,
    fewer rounds, and each against the Leja oracle."""
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=9, count=14)
    nx[2], ny[2] = 1024, 3      # rows longer than a tile, few of them
    nx[3], ny[3] = 2, 200       # two columns: both edge points of the strip
    hx, hy = 1.0 / (nx + 1.0), 1.0 / (ny + 1.0)
    tol = 1e-10 if dtype == "f64" else 1e-7
    bar = TOL_F64 if dtype == "f64" else TOL_F32
    res = {}
    for pairs in (False, True):
        b = E.Batch(nx, ny, hx, hy, tau, tol=tol, dtype=dtype)
        b.set_pairs(pairs)
        assert b.pairs == pairs
        v_all = synth.uniform_vector(b.total_length, 21)
        y = torch.zeros(b.total_length, dtype=torch.float64, device="cuda:0")
        b.prepare()
        print(f"batch pairs={pairs} {dtype}", flush=True)
        b.launch(T(v_all), y)
        stats, rounds = b.results()
        res[pairs] = (N(y), stats, rounds)
    want = leja_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, "dirichlet0", tol)
    (y1, st1, r1), (y2, st2, r2) = res[False], res[True]
    assert r2 < r1
    for i, (yo, sto) in enumerate(want):
        sl = slice(int(b.offsets[i]), int(b.offsets[i]) + int(nx[i] * ny[i]))
        assert relerr(y1[sl], yo) <= bar, (i, relerr(y1[sl], yo))
        assert relerr(y2[sl], yo) <= bar, (i, relerr(y2[sl], yo))
        assert abs(st2[i]["degree_last"] - st1[i]["degree_last"]) <= 1
        assert st1[i]["substeps"] == st2[i]["substeps"]
        extra = st2[i]["newton_steps"] - st1[i]["newton_steps"]
        assert -st1[i]["substeps"] <= extra <= 2 * st1[i]["substeps"], (i, extra)


def test_batch_degree_bound_with_pairs(E):
    """m_max = 12 with two products per round: pairs while j + 2 <= m_max,
    then one single product to m = 12.  Instances whose degree (oracle, same
    tol) is at most 11 converge and match the oracle; those needing 14 or
    more report EXPI_ENOTCONV after exactly m_max products; the same with
    one product per round."""
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=9, count=14)
    res = {}
    for pairs in (True, False):
        b = E.Batch(nx, ny, hx, hy, tau, tol=1e-10, dtype="f64", params=E.LejaParams(m_max=12))
        b.set_pairs(pairs)
        v_all = synth.uniform_vector(b.total_length, 21)
        y = torch.zeros(b.total_length, dtype=torch.float64, device="cuda:0")
        b.prepare()
        print(f"batch m_max 12 pairs={pairs}", flush=True)
        b.launch(T(v_all), y)
        stats, _ = b.results(check_status=False)
        res[pairs] = (N(y), stats)
    want = leja_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, "dirichlet0", 1e-10)
    n_ok = n_fail = 0
    for pairs, (yy, stats) in res.items():
        for i, (yo, sto) in enumerate(want):
            st = stats[i]
            if sto.substeps == 1 and sto.degrees[0] <= 11:
                sl = slice(int(b.offsets[i]), int(b.offsets[i]) + int(nx[i] * ny[i]))
                assert st["status"] == 0 and st["degree_max"] <= 12, (pairs, i, st)
                assert relerr(yy[sl], yo) <= TOL_F64, (pairs, i, relerr(yy[sl], yo))
                n_ok += 1
            elif min(sto.degrees) >= 14:
                assert st["status"] == -4, (pairs, i, st)       # EXPI_ENOTCONV
                assert st["newton_steps"] == 12, (pairs, i, st)  # the first substep stops at m_max
                n_fail += 1
    assert n_ok >= 4 and n_fail >= 16


def test_batch_coef_and_tiles(E):
    """A non-unit coefficient and several tile settings give the oracle's result."""
    nx, ny, hx, hy, tau = batch_case(seed=5, count=7)
    ref = None
    for waves, march in ((4, 8), (2, 16), (1, 4), (8, 64)):
        import torch
        b = E.Batch(nx, ny, hx, hy, tau, coef=0.35, tol=1e-10, dtype="f64")
        b.set_tiles(waves, march)
        v_all = synth.uniform_vector(b.total_length, 2)
        y = torch.zeros(b.total_length, dtype=torch.float64, device="cuda:0")
        b.prepare()
        print(f"batch tiles {waves}x{march}", flush=True)
        b.launch(T(v_all), y)
        stats, _ = b.results()
        if ref is None:
            ref = leja_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, "dirichlet0", 1e-10, coef=0.35)
        yy = N(y)
        for i, (yo, _) in enumerate(ref):
            n = int(nx[i] * ny[i])
            assert relerr(yy[b.offsets[i]:b.offsets[i] + n], yo) <= TOL_F64, (waves, march, i)


def test_batch_larger_grids_against_sine_modes(E):
    """Sizes up to 300^2 and time steps from the cfg range (several substeps)
    against the closed form, FP64 and FP32 storage."""
    nx = np.array([300, 257, 128, 64, 191, 96])
    ny = nx.copy()
    h = 1.0 / (nx + 1.0)
    tau = np.array([3e-4, 1e-5, 1e-3, 5e-4, 1e-4, 9e-4])
    for dtype, bar in (("f64", 1e-9), ("f32", 2e-5)):
        b, v_all, yy, stats, _ = run(E, nx, ny, h, h, tau, tol=1e-10 if dtype == "f64" else 1e-7,
                                     dtype=dtype)
        for i in range(len(nx)):
            n = int(nx[i] * ny[i])
            v = v_all[b.offsets[i]:b.offsets[i] + n]
            want = O.dirichlet_box_phi(1, (int(nx[i]), int(ny[i])), (h[i], h[i]), tau[i], v)
            got = yy[b.offsets[i]:b.offsets[i] + n]
            assert relerr(got, want) <= bar, (dtype, i, relerr(got, want))
        assert max(s["substeps"] for s in stats) > 1


def test_batch_tau_zero_and_single_instance(E):
    """phi_1(0) v = v exactly in FP64 (the divided differences beyond d_0 vanish)."""
    nx, ny = np.array([50]), np.array([37])
    h = 1.0 / (nx + 1.0)
    b, v_all, yy, stats, rounds = run(E, nx, ny, h, h, np.array([0.0]), dtype="f64")
    n = 50 * 37
    assert np.array_equal(yy[:n], v_all[:n])
    assert stats[0]["status"] == 0 and stats[0]["degree_last"] == 2
    assert rounds == 3   # first product, second product (stop), update


def test_batch_round_graph_replays_match_eager(E):
    """Three replays of the captured graph, with eager work and syncs in
    between, each equal to the eager run bit for bit."""
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=3, count=20)
    b = E.Batch(nx, ny, hx, hy, tau, tol=1e-8, dtype="f32")
    v = T(synth.uniform_vector(b.total_length, 5))
    y_eager = torch.zeros_like(v)
    b.prepare()
    b.launch(v, y_eager)
    s_eager, r_eager = b.results()
    y = torch.zeros_like(v)
    b.capture(v, y)
    # rounds = 0 after an eager solve: its round count with a margin, not the bound
    assert b.graph_rounds == min(r_eager + r_eager // 64 + 8, b.max_rounds)
    assert b.graph_rounds < b.max_rounds
    mask = torch.zeros(b.total_length, dtype=torch.bool, device=v.device)
    for i in range(b.count):
        mask[int(b.offsets[i]):int(b.offsets[i]) + int(nx[i] * ny[i])] = True
    for rep in range(3):
        y.fill_(float("nan"))
        scratch = torch.randn(1 << 20, device=v.device).sum()   # eager work in between
        torch.cuda.synchronize()
        print(f"batch graph replay {rep}", flush=True)
        b.replay()
        torch.cuda.synchronize()
        s_rep, r_rep = b.results()
        assert r_rep == r_eager
        assert torch.equal(y[mask], y_eager[mask]), rep
        assert [s["newton_steps"] for s in s_rep] == [s["newton_steps"] for s in s_eager]
        del scratch


def test_batch_short_graph_leaves_instances_unfinished(E):
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=4, count=5)
    b = E.Batch(nx, ny, hx, hy, tau, tol=1e-8, dtype="f64")
    v = T(synth.uniform_vector(b.total_length, 1))
    y = torch.zeros_like(v)
    b.prepare()
    b.capture(v, y, rounds=3)
    assert b.graph_rounds == 3
    b.replay()
    torch.cuda.synchronize()
    stats, rounds = b.results(check_status=False)
    assert rounds == 3
    assert all(s["status"] != 0 for s in stats)
    with pytest.raises(RuntimeError, match="did not finish"):
        b.results()
    # the eager launch afterwards still solves everything
    b.launch(v, y)
    stats, _ = b.results()
    assert all(s["status"] == 0 for s in stats)


def test_batch_rejects_bad_arguments(E):
    import torch
    nx, ny, hx, hy, tau = batch_case(seed=6, count=3)
    b = E.Batch(nx, ny, hx, hy, tau, dtype="f64")
    v = T(synth.uniform_vector(b.total_length + 1, 1))
    y = torch.zeros_like(v)
    with pytest.raises(RuntimeError, match="prepare"):
        b.launch(v[:-1], y[:-1])
    b.prepare()
    with pytest.raises(RuntimeError, match="overlaps"):
        b.launch(v[:-1], v[1:])
    with pytest.raises(RuntimeError, match="aligned"):
        b.launch(v[1:], y[:-1])
    with pytest.raises(RuntimeError, match="overlaps"):
        b.launch_persistent(v[:-1], v[1:])


def test_batch_autotune_picks_a_candidate_and_caches(E, tmp_path):
    import torch
    from paper_1309_4616_amd import autotune
    nx, ny, hx, hy, tau = batch_case(seed=8, count=6)
    b = E.Batch(nx, ny, hx, hy, tau, tol=1e-10, dtype="f64")
    v_all = synth.uniform_vector(b.total_length, 3)
    v = T(v_all)
    y = torch.zeros_like(v)
    path = str(tmp_path / "tiles.json")
    print("batch autotune", flush=True)
    entry = autotune.tune_batch(b, v, y, reps=1, path=path)
    cands = [tuple(c) for c, _ in entry["candidates"]]
    assert len(cands) == 12 and tuple(entry["tiles"]) in cands
    assert b.tiles() == tuple(entry["tiles"])
    assert entry["ms"] == min(t for _, t in entry["candidates"])
    # the tuned batch is prepared and solves correctly
    y.zero_()
    b.launch(v, y)
    b.results()
    want = leja_oracle(nx, ny, hx, hy, tau, v_all, b.offsets, "dirichlet0", 1e-10)
    yy = N(y)
    for i, (yo, _) in enumerate(want):
        n = int(nx[i] * ny[i])
        assert relerr(yy[b.offsets[i]:b.offsets[i] + n], yo) <= TOL_F64
    # a second batch with the same table takes the cached setting without timing
    b2 = E.Batch(nx, ny, hx, hy, tau, tol=1e-10, dtype="f64")
    assert autotune.tune_batch(b2, v, y, path=path) == entry
    assert b2.tiles() == tuple(entry["tiles"])
