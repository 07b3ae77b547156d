"""GPU parity at full size: the 256^3 reaction-diffusion step against the oracle.

The exponential Euler step of eq. (2) on the 256^3 cell-centred grid (the
benchmark's workload: zero-flux boundaries, a = 1 + 0.5 sin 2 pi x sin 2 pi y
sin 2 pi z, Gaussian bump plus noise, tau = 1e-5), computed by the HIP library
in the launch configuration the benchmark times (pair sweeps, FP64), compared
element by element with the FP64 oracle on the assembled 256^3 operator
(about 1.2e8 stored entries, 7 GB of host memory, some 30 s of CPU).  The
single-product kernels on the same step are compared too, and so is the
FP32-storage step.  A 100-step trajectory on the 64^3 grid runs against the
oracle step by step.

Also: the pair sweep's multi-segment march (a workgroup whose chunk of
(row tile, plane) units is longer than one segment of planes), forced by a
grid with 65536 planes, against the oracle.

And: the start vector fused into the first pair sweep against the separate
start sweep on the 256^3 step; the batched workload (256 uneven 2D problems)
against the sine-mode closed form, with the persistent launch equal to the
rounds bit for bit.
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


def rd_op(E, n, amp=0.5):
    coef = synth.sine_coefficient(n, amp)
    h = 1.0 / n
    op = E.StencilOp((n, n, n), (h, h, h), "neumann0",
                     coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))
    return op, coef


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_expeuler_256_step_matches_oracle_elementwise(E):
    import torch
    n = 256
    tau = 1e-5
    op, coef = rd_op(E, n)
    u0 = synth.gaussian_bump_3d(n, seed=0)
    print("256^3 step: GPU pair sweeps (f64), single products (f64), f32 storage", flush=True)
    u = T(u0)
    st = E.expeuler_step(op, tau, u, tol=1e-10)
    got = N(u)
    u.copy_(T(u0))
    ss = E.expeuler_step(op, tau, u, tol=1e-10, params=E.LejaParams(pairs=False))
    got_single = N(u)
    u.copy_(T(u0))
    E.expeuler_step(op, tau, u, tol=1e-8, dtype="f32")
    got32 = N(u)
    del u
    torch.cuda.empty_cache()
    assert st["pair_launches"] >= 1 and ss["pair_launches"] == 0
    print("256^3 step: oracle (assembly, interval, step)", flush=True)
    A = O.stencil_matrix((n, n, n), (1.0 / n,) * 3, "neumann0", coef=coef.field())
    a, b = O.gershgorin_interval(A)
    uo, sto = I.expeuler_step(A, tau, u0, 1e-10, interval=(a, b))
    del A
    assert st["interval_a"] == pytest.approx(a, rel=1e-13)
    assert abs(st["degree_last"] - sto.degrees[-1]) <= 1
    e_state, e_inc = relerr(got, uo), relerr(got - u0, uo - u0)
    e_single = relerr(got_single - u0, uo - u0)
    e32 = relerr(got32, uo)
    print(f"256^3 step vs oracle: state {e_state:.2e}, increment {e_inc:.2e}, "
          f"single products increment {e_single:.2e}, f32 storage state {e32:.2e}", flush=True)
    assert e_state <= TOL_F64
    # the increment tau phi_1(tau A) F(u0) alone, which the state would hide
    assert e_inc <= TOL_F64
    assert e_single <= TOL_F64
    assert relerr(got - u0, got_single - u0) <= 1e-12
    # FP32 storage of the Newton vectors (the state's error floor, not tol)
    assert e32 <= 1e-6
    # mass identity under zero-flux boundaries
    g = u0 - u0 ** 3
    assert abs(got.sum() - (u0.sum() + tau * g.sum())) <= 1e-9 * np.abs(u0).sum()


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_expeuler_64_hundred_steps_match_oracle(E):
    """The 3D workload's 100 steps on the 64^3 grid (tau scaled to keep
    tau (b - a) of the 256^3 grid at 1e-5), every step against the oracle."""
    n = 64
    op, coef = rd_op(E, n)
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=coef.field())
    a, b = O.gershgorin_interval(A)
    tau = 1e-5 * (256 / n) ** 2
    u0 = synth.gaussian_bump_3d(n, seed=0)
    u = T(u0)
    uo = u0.copy()
    worst = worst_inc = 0.0
    for step in range(100):
        prev = uo.copy()
        E.expeuler_step(op, tau, u, tol=1e-10)
        uo, _ = I.expeuler_step(A, tau, uo, 1e-10, interval=(a, b))
        got = N(u)
        e, ei = relerr(got, uo), relerr(got - prev, uo - prev)
        worst, worst_inc = max(worst, e), max(worst_inc, ei)
        assert e <= TOL_F64, (step, e)
    print(f"64^3, 100 steps: worst state error {worst:.2e}, worst increment error {worst_inc:.2e}")
    # increments compared against the oracle's own previous state carry the
    # accumulated state difference; they stay far below the tolerance
    assert worst_inc <= 1e-8


def test_pair_sweep_multi_segment_march(E):
    """65536 planes of 2 x 6 points: one row tile, 65536 (row tile, plane)
    units, so on a 256-CU part each workgroup's chunk holds 256 planes,
    more than one segment (248 planes), and the march refills its plane
    table and restarts its rings mid-chunk."""
    shape = (2, 6, 65536)
    h = (1.0 / 2, 1.0 / 6, 1.0 / 65536)
    tabs = [np.cos(2 * np.pi * (np.arange(s) + 0.5) / s) for s in shape]
    c0, c1 = 1.0, 0.45
    fld = c0 + c1 * ((tabs[2][:, None, None] * tabs[1][None, :, None]) * tabs[0][None, None, :])
    for bc in ("neumann0", "dirichlet0"):
        op = E.StencilOp(shape, h, bc, coef=("separable", c0, c1, *tabs))
        A = O.stencil_matrix(shape, h, bc, coef=fld.reshape(-1))
        a, b = O.gershgorin_interval(A)
        tau = 12.0 / (b - a)
        v = synth.uniform_vector(A.shape[0], 11)
        print(f"multi-segment march {shape} {bc}", flush=True)
        y, st = E.phi_action(op, 1, tau, T(v), tol=1e-10, params=E.LejaParams(profile=1))
        ys, _ = E.phi_action(op, 1, tau, T(v), tol=1e-10, params=E.LejaParams(pairs=False))
        yo, so = I.phi_action(A, 1, tau, v, 1e-10, interval=(a, b))
        assert st["timed_pairs"] >= 1
        assert relerr(N(y), yo) <= TOL_F64, (bc, relerr(N(y), yo))
        assert relerr(N(y), N(ys)) <= 1e-12


def test_expeuler_512_fp32_pairs_equal_singles(E):
    """The 3D workload at 512^3 with FP32 storage (the bench leg beyond the
    MALL, tau scaled to keep tau (b - a) of 256^3): pair sweeps on rows of 512
    points (four waves per row, two output rows per workgroup) against
    single products, element by element, to FP32 rounding; no oracle at this
    size (its operator would need about 60 GB of host memory)."""
    import torch
    n = 512
    op, _ = rd_op(E, n)
    u0 = torch.as_tensor(synth.gaussian_bump_3d(n, seed=0), device="cuda:0")
    tau = 1e-5 * (256 / n) ** 2
    up, us = u0.clone(), u0.clone()
    print("512^3 FP32 Euler step, pairs then singles", flush=True)
    sp = E.expeuler_step(op, tau, up, tol=1e-8, dtype="f32", params=E.LejaParams(profile=True))
    ss = E.expeuler_step(op, tau, us, tol=1e-8, dtype="f32", params=E.LejaParams(pairs=False, profile=True))
    assert sp["timed_pairs"] >= 1 and ss["timed_pairs"] == 0
    assert abs(sp["degree_last"] - ss["degree_last"]) <= 1
    d = ((up - us).norm() / (us - u0).norm()).item()
    assert d <= 1e-5, d
    del op, u0, up, us
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_pair_sweep_at_its_size_limit(E):
    """Pair sweeps address a vector with 32-bit byte offsets, so they take
    grids of FP64 vectors below 2^31 bytes.  A grid just below the limit
    (512 x 512 x 1022 points, 2.14 GB per vector) runs pair sweeps and gives
    the single products' result to rounding; one at the limit (512 x 512 x
    1024, 2^31 bytes) runs single products only and still converges."""
    import torch
    gen = torch.Generator(device="cuda:0")
    for nz, pairs_expected in ((1022, True), (1024, False)):
        shape = (512, 512, nz)
        h = (1.0 / 512, 1.0 / 512, 1.0 / nz)
        op = E.StencilOp(shape, h, "neumann0", coef=1.0)
        n = 512 * 512 * nz
        gen.manual_seed(5)
        v = torch.rand(n, generator=gen, device="cuda:0", dtype=torch.float64) - 0.5
        a, b = op.interval()
        tau = 6.0 / (b - a)
        print(f"size limit: {shape}, {8 * n} bytes per vector", flush=True)
        yp, sp = E.phi_action(op, 1, tau, v, tol=1e-12, params=E.LejaParams(profile=True))
        assert (sp["timed_pairs"] >= 1) == pairs_expected
        if pairs_expected:
            ys, ss = E.phi_action(op, 1, tau, v, tol=1e-12, params=E.LejaParams(pairs=False, profile=True))
            assert ss["timed_pairs"] == 0 and ss["degree_last"] == sp["degree_last"]
            d = ((yp - ys).abs().max() / ys.abs().max()).item()
            assert d <= 1e-12, d
            del ys
        assert sp["converged"] == 1
        del op, v, yp
        torch.cuda.empty_cache()


def test_expeuler_256_fused_start_equals_separate(E):
    """At full size (256^3, the benchmark's operator and state), the start
    vector fused into the first pair sweep gives the separate start sweep's
    step to rounding, in FP64 and with FP32 storage (the configuration the
    benchmark times fuses whenever the previous step stopped at an odd
    degree)."""
    import torch
    n = 256
    op, _ = rd_op(E, n)
    u0 = torch.as_tensor(synth.gaussian_bump_3d(n, seed=0), device="cuda:0")
    for dtype, bar in (("f64", 1e-12), ("f32", 1e-5)):
        res = {}
        for fs in (1, 2):
            u = u0.clone()
            print(f"256^3 {dtype} fuse_start={fs}", flush=True)
            st = E.expeuler_step(op, 1e-5, u, tol=1e-8, dtype=dtype, params=E.LejaParams(fuse_start=fs))
            assert st["fused_starts"] == (1 if fs == 2 else 0)
            res[fs] = u - u0
        d = ((res[2] - res[1]).norm() / res[1].norm()).item()
        assert d <= bar, (dtype, d)
    del op, u0, res
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.timeout(600)
# FP64 bar: the stop test bounds each substep's error by about tol, and the
# largest instances take up to 85 substeps
@pytest.mark.parametrize("dtype,tol,bar", [("f32", 1e-8, 5e-6), ("f64", 1e-10, 1e-8)])
def test_batched_256_problems_against_sine_modes(E, dtype, tol, bar):
    """The batched workload at full size (256 uneven 2D Dirichlet problems,
    sides 64..1024; FP32 storage at tol 1e-8, and FP64 at tol 1e-10): every
    instance against the FP64 sine-mode closed form, the persistent launch
    bitwise equal to the rounds.  At this size the waves take many tiles
    each, one after another."""
    import torch
    inst = synth.batched_instances(256, seed=0)
    ns = np.array([it.n for it in inst])
    taus = np.array([it.tau for it in inst])
    h = 1.0 / (ns + 1.0)
    b = E.Batch(ns, ns, h, h, taus, bc="dirichlet0", tol=tol, dtype=dtype)
    v_host = np.zeros(b.total_length)
    for i, it in enumerate(inst):
        o = int(b.offsets[i])
        v_host[o:o + it.n * it.n] = synth.uniform_vector(it.n * it.n, it.seed)
    v = torch.as_tensor(v_host, device="cuda:0")
    y = torch.zeros_like(v)
    b.prepare()
    print(f"batched 256 {dtype}: rounds", flush=True)
    b.launch(v, y)
    stats, rounds = b.results()
    yy = y.cpu().numpy()
    worst = 0.0
    for i, it in enumerate(inst):
        o, n2 = int(b.offsets[i]), it.n * it.n
        want = O.dirichlet_box_phi(1, (it.n, it.n), (h[i], h[i]), it.tau, v_host[o:o + n2])
        e = relerr(yy[o:o + n2], want)
        worst = max(worst, e)
        assert e <= bar, (i, it.n, e)
        assert stats[i]["status"] == 0
    print(f"batched 256: {rounds} rounds, worst error {worst:.2e}", flush=True)
    y2 = torch.zeros_like(v)
    print("batched 256: persistent", flush=True)
    b.launch_persistent(v, y2)
    _, r2 = b.results()
    assert r2 == rounds
    mask = torch.zeros(b.total_length, dtype=torch.bool, device=v.device)
    for i, it in enumerate(inst):
        mask[int(b.offsets[i]):int(b.offsets[i]) + it.n * it.n] = True
    assert torch.equal(y2[mask], y[mask])
