"""GPU tests of the step-selector network and the learned mode.

* forward, backward and Adam kernels against the float64 oracle (oracle.mlp);
* the learned mode on held-out exponential Euler steps of the 3D
  reaction-diffusion problem: same accuracy as the plain method, with the
  network's degree prediction replacing most stop tests;
* the gain of the learned substep count on steps whose size changes from
  step to step (tau (b - a) from 20 to 800, so the plain method has no
  degree hint and often several substeps): fewer products and less time at
  the same tolerance, with device and host features equal.
"""
import math

import numpy as np
import pytest

import synth
from oracle import integrators as I
from oracle import mlp as omlp
from oracle import operators as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E(device):
    import paper_1309_4616_amd as E
    E.lib()
    return E


def unpack(vec, H):
    """Packed W1 b1 W2 b2 W3 b3 -> the oracle's dict."""
    o = 0
    out = {}
    for name, shape in (("W1", (H, 8)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("W3", (2, H)), ("b3", (2,))):
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


@pytest.mark.parametrize("H", [16, 64])
def test_mlp_kernels_match_oracle(E, H):
    import torch
    rng = np.random.default_rng(H)
    net = E.selector.Net(H, seed=3)
    p64 = unpack(net.params.double().cpu().numpy(), H)
    for k in ("b1", "b2", "b3"):
        p64[k] = rng.uniform(-0.3, 0.3, size=p64[k].shape)
    net.params.copy_(torch.as_tensor(pack(p64), dtype=torch.float32))
    p64 = unpack(net.params.double().cpu().numpy(), H)   # what the device holds
    n = 37
    x = rng.standard_normal((n, 8))
    t = rng.standard_normal((n, 2))
    xt = torch.as_tensor(x, dtype=torch.float32, device="cuda:0")
    tt = torch.as_tensor(t, dtype=torch.float32, device="cuda:0")
    x32 = xt.double().cpu().numpy()
    t32 = tt.double().cpu().numpy()
    o_ref, cache = omlp.forward(p64, x32)
    g, loss, out = net.grad(xt, tt, kappa=3.0)
    assert np.allclose(out.double().cpu().numpy(), o_ref, rtol=1e-5, atol=1e-5)
    assert loss.item() == pytest.approx(omlp.loss(o_ref, t32, 3.0), rel=1e-5)
    g_ref = pack(omlp.backward(p64, cache, o_ref, t32, kappa=3.0))
    gg = g.double().cpu().numpy()
    scale = np.abs(g_ref).max()
    assert np.max(np.abs(gg - g_ref)) <= 1e-4 * scale
    # Adam: three steps with the same gradient against the oracle's update
    m = {k: np.zeros_like(v) for k, v in p64.items()}
    v = {k: np.zeros_like(w) for k, w in p64.items()}
    gd = unpack(gg, H)
    pr = {k: w.copy() for k, w in p64.items()}
    for step in range(1, 4):
        net.adam(g, lr=1e-2)
        omlp.adam_step(pr, gd, m, v, step, lr=1e-2)
    assert np.allclose(net.params.double().cpu().numpy(), pack(pr), rtol=1e-5, atol=1e-6)


def rd_op(E, n, amp):
    coef = synth.sine_coefficient(n, amp)
    h = 1.0 / n
    return E.StencilOp((n, n, n), (h, h, h), "neumann0",
                       coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))


def log_plain(E, n, amps, steps, tau, tol, seed0):
    """Run plain exponential Euler trajectories; return features, targets, stats."""
    import torch
    X, Y, runs = [], [], []
    for k, amp in enumerate(amps):
        op = rd_op(E, n, amp)
        u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=seed0 + k), device="cuda:0")
        for _ in range(steps):
            st = E.expeuler_step(op, tau, u, tol=tol)
            X.append(E.selector.features(st, tau))
            Y.append(E.selector.targets(st))
            runs.append(st)
    return np.array(X), np.array(Y), runs


def test_learned_selector_on_held_out_steps(E):
    import torch
    n = 40
    tau = 1e-5 * (256 / n) ** 2     # same stiffness tau*(b-a) as the 256^3 grid at 1e-5
    tol = 1e-8
    amps = synth.diffusivity_amplitudes(8, seed=7)
    X, Y, _ = log_plain(E, n, amps[:6], 12, tau, tol, seed0=100)
    net, norms, hist = E.selector.train(X, Y, hidden=64, epochs=1500, lr=3e-3, seed=0)
    assert hist[-1] < 0.5 * hist[0]
    sel = E.selector.pack(net, norms)
    pred = E.selector.predict(net, norms, X)
    assert np.mean(np.abs(pred[:, 1] - Y[:, 1])) < 1.5      # fits the degrees it saw
    # held-out trajectories: plain vs learned from the same states, each step
    # on fresh operator objects, so that neither method has a degree from an
    # earlier step (the learned mode consults the network only then)
    plain_mv = learned_mv = plain_fin = learned_fin = 0
    for k, amp in enumerate(amps[6:]):
        u0 = torch.as_tensor(synth.gaussian_bump_3d(n, seed=500 + k), device="cuda:0")
        up, ul = u0.clone(), u0.clone()
        params = E.LejaParams(selector=sel, selector_hidden=64)
        for step in range(10):
            sp = E.expeuler_step(rd_op(E, n, amp), tau, up, tol=tol)
            sl = E.expeuler_step(rd_op(E, n, amp), tau, ul, tol=tol, params=params)
            plain_mv += sp["matvecs"]
            learned_mv += sl["matvecs"]
            plain_fin += sp["finalized"]
            learned_fin += sl["finalized"]
            assert sl["pred_degree"] > 0
            # both met the same two-term test at 1e-8: states agree to that level
            d = (ul - up).norm().item() / up.norm().item()
            assert d <= 5e-8, (step, d)
    # the prediction replaces most stop tests; products stay within ~10%
    assert learned_fin < 0.6 * plain_fin
    assert learned_mv <= 1.1 * plain_mv + 2
    print(f"matvecs plain {plain_mv} learned {learned_mv}; stop tests plain {plain_fin} learned {learned_fin}")


def test_learned_mode_matches_oracle(E):
    """The learned mode's result is judged by the same stop test: at tol 1e-10
    it agrees with the oracle like the plain method does."""
    import torch
    n = 24
    tau = 1e-5 * (256 / n) ** 2
    X, Y, _ = log_plain(E, n, [0.3, 0.6, 0.8], 6, tau, 1e-10, seed0=1)
    net, norms, _ = E.selector.train(X, Y, hidden=32, epochs=800, lr=3e-3, seed=1)
    sel = E.selector.pack(net, norms)
    op = rd_op(E, n, 0.5)
    u0 = synth.gaussian_bump_3d(n, seed=9)
    u = torch.as_tensor(u0, device="cuda:0")
    st = E.expeuler_step(op, tau, u, tol=1e-10, params=E.LejaParams(selector=sel, selector_hidden=32))
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=synth.sine_coefficient(n, 0.5).field())
    uo, _ = I.expeuler_step(A, tau, u0, 1e-10)
    got = u.cpu().numpy()
    assert np.linalg.norm(got - uo) / np.linalg.norm(uo) <= 1e-10
    assert st["pred_degree"] > 0


def test_learned_mode_near_l_max_matches_oracle(E):
    """tau (b - a) close to l_max = 100 (one substep, degree about 45 at
    1e-10): the Newton terms still grow past the fourth product, so the
    first stop test after the unreduced products must use the term of the
    product just before it.  Learned mode against the oracle at 1e-10."""
    import torch
    n = 20
    coef = synth.sine_coefficient(n, 0.5)
    A = O.stencil_matrix((n, n, n), (1 / n,) * 3, "neumann0", coef=coef.field())
    a, b = O.gershgorin_interval(A)
    tau = 95.0 / (b - a)
    X, Y, _ = log_plain(E, n, [0.3, 0.5, 0.7], 4, tau, 1e-10, seed0=40)
    net, norms, _ = E.selector.train(X, Y, hidden=32, epochs=800, lr=3e-3, seed=2)
    sel = E.selector.pack(net, norms)
    for seed in (41, 42):
        op = rd_op(E, n, 0.5)          # no degree from an earlier step
        u0 = synth.gaussian_bump_3d(n, seed=seed)
        u = torch.as_tensor(u0, device="cuda:0")
        st = E.expeuler_step(op, tau, u, tol=1e-10,
                             params=E.LejaParams(selector=sel, selector_hidden=32))
        uo, sto = I.expeuler_step(A, tau, u0, 1e-10, interval=(a, b))
        got = u.cpu().numpy()
        assert st["substeps"] == 1 and st["pred_degree"] > 8
        # a stop at m needs the two-term test at m, so the learned loop never
        # stops before the oracle's first m (up to rounding at the threshold)
        assert st["degree_last"] >= sto.degrees[-1] - 1
        assert np.linalg.norm(got - uo) / np.linalg.norm(uo) <= 1e-10
        # the increment alone: the two differ by at most the oracle's own
        # truncation (the stop test holds it to 1e-10 of ||p||)
        assert np.linalg.norm((got - u0) - (uo - u0)) / np.linalg.norm(uo - u0) <= 1e-9


def test_learned_substeps_gain_on_variable_step_sizes(E):
    """Labels: for each logged step, the substep count with the fewest
    products among those that converge (selector.best_label).  On held-out
    steps the learned mode must take at least 20% fewer products and less
    time than the plain method, both against a tol 1e-13 reference within
    the error the tolerance allows, and the selector kernel's features must
    equal the host's."""
    import torch
    n = 32
    tol = 1e-8
    rng = np.random.default_rng(11)
    amps = synth.diffusivity_amplitudes(7, seed=12)

    def draw_tau(a, b):
        return math.exp(rng.uniform(math.log(20.0), math.log(800.0))) / (b - a)

    X, Y = [], []
    for k, amp in enumerate(amps[:5]):
        op = rd_op(E, n, amp)
        a, b = op.interval()
        u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=300 + k), device="cuda:0")
        for _ in range(12):
            tau = draw_tau(a, b)
            L = tau * (b - a)

            def forced(s, u=u, tau=tau, L=L, op=op):
                try:
                    return E.expeuler_step(op, tau, u.clone(), tol=tol, params=E.LejaParams(
                        l_max=E.selector.forced_substeps_l_max(L, s), max_retries=0))
                except E.ExpiError:
                    return None
            st = E.expeuler_step(op, tau, u, tol=tol)
            lab, _ = E.selector.best_label(forced, L, st["substeps"], st)
            X.append(E.selector.features(st, tau))
            Y.append(lab)
    net, norms, hist = E.selector.train(np.array(X), np.array(Y), hidden=64, epochs=2000, lr=3e-3,
                                        kappa=1.5, seed=0)
    sel = E.selector.pack(net, norms)
    feat = torch.zeros(8, dtype=torch.float32, device="cuda:0")
    lp = E.LejaParams(selector=sel, selector_hidden=64, selector_features=feat)
    mv = {"plain": 0, "learned": 0}
    ms = {"plain": 0.0, "learned": 0.0}
    import time
    for k, amp in enumerate(amps[5:]):
        # one operator object per method (each keeps its own degree hints)
        op, op_l, op_r = rd_op(E, n, amp), rd_op(E, n, amp), rd_op(E, n, amp)
        a, b = op.interval()
        u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=700 + k), device="cuda:0")
        for step in range(10):
            tau = draw_tau(a, b)
            ref = u.clone()
            E.expeuler_step(op_r, tau, ref, tol=1e-13)
            ul = u.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sp = E.expeuler_step(op, tau, u, tol=tol)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sl = E.expeuler_step(op_l, tau, ul, tol=tol, params=lp)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            mv["plain"] += sp["matvecs"]
            mv["learned"] += sl["matvecs"]
            ms["plain"] += 1e3 * (t1 - t0)
            ms["learned"] += 1e3 * (t2 - t1)
            ep = ((u - ref).norm() / ref.norm()).item()
            el = ((ul - ref).norm() / ref.norm()).item()
            assert ep <= 5e-8 and el <= 5e-8, (step, ep, el)
            assert sl["pred_degree"] > 0
            # the features the selector kernel computed (from the probe at
            # the plain substep count) are the host's, to float32 rounding
            hf = E.selector.features(sp, tau)
            assert np.allclose(feat.cpu().numpy(), hf, rtol=1e-5, atol=1e-6)
    print(f"variable steps: products plain {mv['plain']} learned {mv['learned']}; "
          f"ms plain {ms['plain']:.1f} learned {ms['learned']:.1f}")
    assert mv["learned"] <= 0.8 * mv["plain"]
    assert ms["learned"] < ms["plain"]


def test_learned_mode_follows_plain_loop_once_a_degree_is_known(E):
    """With one substep allowed (tau (b - a) well below l_max) and a degree
    known from an earlier step of the same substep length, the network could
    change nothing: the learned mode runs the plain loop with that degree,
    launch for launch, and its result equals the plain method's bitwise."""
    import torch
    n = 24
    tau = 1e-5 * (256 / n) ** 2
    X, Y, _ = log_plain(E, n, [0.3, 0.6], 4, tau, 1e-8, seed0=60)
    net, norms, _ = E.selector.train(X, Y, hidden=32, epochs=300, lr=3e-3, seed=3)
    params = E.LejaParams(selector=E.selector.pack(net, norms), selector_hidden=32)
    op_p, op_l = rd_op(E, n, 0.5), rd_op(E, n, 0.5)
    u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=61), device="cuda:0")
    # a fresh operator has no degree: the network decides
    st = E.expeuler_step(rd_op(E, n, 0.5), tau, u.clone(), tol=1e-8, params=params)
    assert st["pred_degree"] > 0
    # one plain step on each operator gives both the same degree
    for op in (op_p, op_l):
        E.expeuler_step(op, tau, u.clone(), tol=1e-8)
    for step in range(3):
        ul = u.clone()
        sp = E.expeuler_step(op_p, tau, u, tol=1e-8)
        sl = E.expeuler_step(op_l, tau, ul, tol=1e-8, params=params)
        assert sl["pred_degree"] == 0
        assert sl["matvecs"] == sp["matvecs"] and sl["degree_last"] == sp["degree_last"]
        assert torch.equal(ul, u), step
