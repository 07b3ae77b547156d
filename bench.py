#!/usr/bin/env python3
"""Throughput of the exponential-integrator hot path on one MI355X.

Workload: exponential Euler steps of the 3D reaction-diffusion problem
u_t = div(a grad u) + u - u^3 on the 256^3 cell-centred grid of the unit cube,
zero-flux (homogeneous Neumann) boundaries, a = 1 + 0.5 sin(2 pi x) sin(2 pi y)
sin(2 pi z), u0 = Gaussian bump (sigma 0.1, centre (1/2,1/2,1/2)) + 0.01 N(0,1)
noise (seed 0), tau = 1e-5, relative tolerance 1e-8.  Each step is one
phi_1(tau A) action (Leja-point Newton interpolation) plus its start vector
and update, all in the HIP library; consecutive Newton products run as pair
sweeps (two products per pass) unless --no-pairs.

A step of the benchmark is one exponential Euler step on the whole grid.
`value` is solved grid points per second (points x steps / wall time) in
FP64; the same run is repeated with FP32 storage of the Newton vectors.
`roofline` covers the dominant kernel (the pair sweep), whose launches are
timed with HIP events on the library's stream during the timed region.
`cpu_baseline` is the FP64 oracle on a bounded sample of the same workload.
Further legs: the learned step selector against the plain loop, the
batched solve of 256 uneven 2D problems, the CSR product, the paper's Table
I-IV kernels, the complex spin-bath case, and the plain method on 2D
Dirichlet Laplacians (128^2, and 8192^2 in FP64 and FP32 storage) with 2D
pair sweeps against single products.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = ("φ1(τA)v throughput: HBM GB/s + grid pts/s at 1e-8 rel err; "
          "learned vs plain")
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per grid point of the fused Newton product:
# read w_j, write w_{j+1}, read and write p (the separable coefficient costs 0)
NEWTON_BYTES_PER_PT = {"f64": 32, "f32": 16}


def step_bytes_per_pt(launches: int, loops: int, fused_starts: int, dt: str) -> int:
    """Algorithmic bytes per point of a run of exponential Euler steps from
    its launch counts: each Newton loop (one per substep) opens with a launch
    that moves three vectors (read r or u, write w and p), every further
    pair sweep or single product reads w and p and writes w and p, each
    start vector not formed inside the opening pair sweep reads u and writes
    r, and each substep's update reads u and p and writes u."""
    s = 8 if dt == "f64" else 4
    opening = 3 * s
    newton = 4 * s
    start = 8 + s
    update = 8 + s + 8
    return ((launches - loops) * newton + loops * (opening + update) +
            (loops - fused_starts) * start)


def counter_traffic(kernel_sub: str):
    """HBM bytes per launch of a kernel from a committed rocprofv3 summary
    under profiles/ (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of
    known size), or None if no summary covers it or its source files have
    changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*.md"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if kernel_sub not in blob.get("kernel", ""):
            continue
        h = hashlib.sha256()
        try:
            for f in blob["source_files"]:
                h.update(open(os.path.join(HERE, f), "rb").read())
        except OSError:
            return None
        if h.hexdigest() != blob.get("source_sha256"):
            return None
        return {"bytes": blob["traffic_bytes_per_launch"], "profile": os.path.relpath(path, HERE)}
    return None


def copy_ceiling():
    """A plain device copy (torch's copy kernel: one read and one write of
    every byte) at two sizes: 2 GiB per array, far beyond the 256 MB MALL,
    and 134 MB (one 256^3 float64 vector).  Bytes moved (read + written)
    per second, HIP events around 10 copies after 2 warm-ups: a measured
    ceiling for streaming kernels beside the 8 TB/s peak."""
    import torch
    out = {}
    for label, n in (("2GiB", 1 << 28), ("256^3_f64", 256 ** 3)):
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        out[label] = {"bytes_moved": 16 * n, "us": 1e3 * ms, "gbs": 16 * n / (ms * 1e-3) / 1e9}
        del src, dst
    torch.cuda.empty_cache()
    return out


def run_gpu(args, dtype: str, n: int = None, tau: float = None, steps: int = None, warmup: int = None):
    import torch
    import paper_1309_4616_amd as E
    import synth

    n = n or args.n
    tau = tau or args.tau
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    h = 1.0 / n
    coef = synth.sine_coefficient(n, 0.5)
    op = E.StencilOp((n, n, n), (h, h, h), "neumann0",
                     coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))
    u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=0), device="cuda:0")
    ws = op.workspace(dtype)
    # the library's autotuner picks the single-product tiles and whether the
    # pair sweep (the dominant kernel) runs, by timing both on this operator
    from paper_1309_4616_amd import autotune
    tuned = autotune.tune(op, dtype, reps=3, use_cache=False)
    # every fourth timed step runs with HIP events around each of its Newton
    # launches (profile=1); the others without (events around every launch
    # of every step would cost about 4% of the step).  The launch average is
    # over all Newton launches of those steps: single launches vary by +-15%
    # within a step, the first after a loop's opening among the slowest.
    params = E.LejaParams(profile=0, pairs=not args.no_pairs)
    params_timed = E.LejaParams(profile=1, pairs=not args.no_pairs)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        E.expeuler_step(op, tau, u, tol=args.tol, dtype=dtype, params=params, ws=ws)
    torch.cuda.synchronize()
    matvecs = newton = timed = pairs = 0
    pair_launches = single_launches = loops = fused = 0
    newton_ms = pair_ms = 0.0
    degrees = []
    t0 = time.perf_counter()
    for i in range(steps):
        st = E.expeuler_step(op, tau, u, tol=args.tol, dtype=dtype, params=params_timed if i % 4 == 0 else params,
                             ws=ws)
        matvecs += st["matvecs"]
        newton += st["newton_steps"]
        timed += st["timed_products"]
        newton_ms += st["newton_ms"]
        pairs += st["timed_pairs"]
        pair_ms += st["pair_ms"]
        pair_launches += st["pair_launches"]
        single_launches += st["single_launches"]
        loops += st["substeps"]
        fused += st["fused_starts"]
        degrees.append(st["degree_last"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del stream
    pts = n ** 3
    singles = timed - 2 * pairs          # timed single products (sampled)
    bytes_total = pts * step_bytes_per_pt(pair_launches + single_launches, loops, fused, dtype)
    per_launch = NEWTON_BYTES_PER_PT[dtype] * pts
    single_us = 1e3 * (newton_ms - pair_ms) / max(singles, 1)
    pair_us = 1e3 * pair_ms / max(pairs, 1)
    return {
        "wall_s": wall,
        "value": pts * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "matvecs_per_step": matvecs / steps,
        "newton_per_step": newton / steps,
        "degrees": sorted(set(degrees)),
        "point_products_per_s": pts * matvecs / wall,
        "step_gbs": bytes_total / wall / 1e9,
        "pairs_per_step": pair_launches / steps,
        "singles_per_step": single_launches / steps,
        "fused_starts_per_step": fused / steps,
        "timed_launches": pairs + singles,
        "pair_avg_us": pair_us if pairs else None,
        "pair_gbs": per_launch / (pair_us * 1e-6) / 1e9 if pairs else None,
        "single_avg_us": single_us if singles else None,
        "single_gbs": per_launch / (single_us * 1e-6) / 1e9 if singles else None,
        "u_checksum": float(u.double().sum().item()),
        "autotune": {"pairs": tuned["pairs"], "single_tiles": tuned["tiles"], "single_us": tuned["us"],
                     "pair_us": next((t for c, t in tuned["candidates"] if c == [0, 0, 2]), None)},
    }


def run_learned(args):
    """Learned vs plain (the step-selector workload): exponential Euler steps
    of the same 256^3 problem over trajectories whose diffusivity amplitude
    is drawn from [0.1, 0.9] (seeded) and whose step size changes from step
    to step, tau (b - a) log-uniform in [10, 1000] (so the plain method has
    no degree hint and takes up to 10 substeps).  `train_steps` logged plain
    steps, each labelled with the substep count that needed the fewest
    products among those that converge, train the network on the GPU with
    the library's kernels; `eval_steps` held-out steps then run both ways
    from the same states at the same tolerance, every fifth one also against
    a tol 1e-13 reference.  The same network is also evaluated on held-out
    steps of fixed size tau = 1e-5 (tau (b - a) about 12)."""
    import numpy as np
    import torch
    import paper_1309_4616_amd as E
    import synth

    n = args.n
    h = 1.0 / n
    per = 100
    n_train = max(1, args.train_steps // per)
    n_eval = max(1, args.eval_steps // per)
    amps = synth.diffusivity_amplitudes(n_train + n_eval, seed=2024)
    rng = np.random.default_rng(np.random.SeedSequence(77))

    def make_op(amp):
        coef = synth.sine_coefficient(n, float(amp))
        return E.StencilOp((n, n, n), (h, h, h), "neumann0",
                           coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))

    def draw_tau(a, b):
        return float(np.exp(rng.uniform(np.log(10.0), np.log(1000.0)))) / (b - a)

    X, Y = [], []
    t0 = time.perf_counter()
    for k in range(n_train):
        op = make_op(amps[k])
        a, b = op.interval()
        ws = op.workspace("f64")
        u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=1000 + k), device="cuda:0")
        for _ in range(min(per, args.train_steps)):
            tau = draw_tau(a, b)
            L = tau * (b - a)

            def forced(s, u=u, tau=tau, L=L, op=op, ws=ws):
                try:
                    return E.expeuler_step(op, tau, u.clone(), tol=args.tol, ws=ws, params=E.LejaParams(
                        l_max=E.selector.forced_substeps_l_max(L, s), max_retries=0))
                except E.ExpiError:
                    return None
            st = E.expeuler_step(op, tau, u, tol=args.tol, ws=ws)
            lab, _ = E.selector.best_label(forced, L, st["substeps"], st)
            X.append(E.selector.features(st, tau))
            Y.append(lab)
        del op, ws
    log_s = time.perf_counter() - t0
    X, Y = np.array(X), np.array(Y)
    t0 = time.perf_counter()
    net, norms, hist = E.selector.train(X, Y, hidden=64, epochs=2000, lr=3e-3, kappa=args.sel_kappa, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    sel = E.selector.pack(net, norms)
    lp = E.LejaParams(selector=sel, selector_hidden=64)

    def evaluate(fixed_tau):
        res = {"plain": {"mv": 0, "tests": 0, "t": 0.0, "err": 0.0},
               "learned": {"mv": 0, "tests": 0, "t": 0.0, "err": 0.0}}
        fallbacks = steps = fewer = consulted = 0
        for k in range(n_eval):
            # one operator object per method: each keeps its own degree
            # hints (keyed by the substep length), as a run of that method
            # alone would; the reference at tol 1e-13 has its own too
            ops = {key: make_op(amps[n_train + k]) for key in ("plain", "learned", "ref")}
            op = ops["plain"]
            a, b = op.interval()
            ws = op.workspace("f64")
            u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=5000 + k), device="cuda:0")
            E.expeuler_step(op, fixed_tau or draw_tau(a, b), u.clone(), tol=args.tol, ws=ws)  # warm-up
            for i in range(min(per, args.eval_steps)):
                tau = fixed_tau or draw_tau(a, b)
                ref = None
                if i % 5 == 0:
                    ref = u.clone()
                    E.expeuler_step(ops["ref"], tau, ref, tol=1e-13, ws=ws)
                ul = u.clone()
                for key, uu, params in (("plain", u, None), ("learned", ul, lp)):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    st = E.expeuler_step(ops[key], tau, uu, tol=args.tol, params=params, ws=ws)
                    torch.cuda.synchronize()
                    res[key]["t"] += time.perf_counter() - t1
                    res[key]["mv"] += st["matvecs"]
                    res[key]["tests"] += st["finalized"]
                    if ref is not None:
                        res[key]["err"] = max(res[key]["err"], ((uu - ref).norm() / ref.norm()).item())
                    if key == "learned":
                        consulted += 1 if st["pred_degree"] > 0 else 0
                        fallbacks += 1 if st["fallback"] else 0
                        fewer += 1 if st["substeps"] < s_plain else 0
                    else:
                        s_plain = st["substeps"]
                steps += 1
            del op, ops, ws
        out = {"eval_steps": steps, "fallback_rate": fallbacks / max(steps, 1),
               "steps_with_fewer_substeps": fewer, "steps_network_consulted": consulted}
        for key in ("plain", "learned"):
            out[key] = {"matvecs_per_step": res[key]["mv"] / steps,
                        "stop_tests_per_step": res[key]["tests"] / steps,
                        "ms_per_step": 1e3 * res[key]["t"] / steps,
                        "max_err_vs_tol_1e-13": res[key]["err"]}
        out["matvecs_ratio"] = out["learned"]["matvecs_per_step"] / out["plain"]["matvecs_per_step"]
        out["time_ratio"] = out["learned"]["ms_per_step"] / out["plain"]["ms_per_step"]
        return out

    variable = evaluate(None)
    fixed = evaluate(args.tau)
    return {
        "train_steps": len(X), "hidden": 64, "log_and_label_s": log_s, "train_s": train_s,
        "loss_first_last": [hist[0], hist[-1]], "tol": args.tol,
        "label": "substep count with the fewest products among those that converge",
        "variable_tau": dict(variable, workload="tau (b - a) log-uniform in [10, 1000] per step"),
        "fixed_tau": dict(fixed, workload=f"tau = {args.tau:g} (tau (b - a) about 12)"),
    }


def run_batched(args):
    """The batched workload: `batch_count` independent 2D Dirichlet problems,
    side lengths log-uniform in [64, 1024] and tau uniform in [1e-5, 1e-3]
    (seeded), FP32 storage of the Newton vectors with float64 divided
    differences, norms, stop test and y; solved eagerly (host-enqueued rounds)
    as one replay of the captured round graph, and in one persistent kernel
    launch (directly and as a replayed graph).  Errors per instance are
    against the float64 sine-mode closed form of phi_1(tau A) v."""
    import numpy as np
    import torch
    import paper_1309_4616_amd as E
    import synth
    from oracle import operators as O
    from paper_1309_4616_amd import autotune

    inst = synth.batched_instances(args.batch_count, seed=0)
    ns = np.array([it.n for it in inst])
    taus = np.array([it.tau for it in inst])
    h = 1.0 / (ns + 1.0)
    b = E.Batch(ns, ns, h, h, taus, bc="dirichlet0", tol=args.tol, dtype="f32")
    v_host = np.zeros(b.total_length)
    for i, it in enumerate(inst):
        o = int(b.offsets[i])
        v_host[o:o + it.n * it.n] = synth.uniform_vector(it.n * it.n, it.seed)
    v = torch.as_tensor(v_host, device="cuda:0")
    y = torch.zeros_like(v)
    # tile shape chosen by the library's autotuner (one timed solve per candidate)
    tuned = autotune.tune_batch(b, v, y, reps=1, use_cache=False)
    b.launch(v, y)                      # warm-up (also the eager reference)
    stats, rounds = b.results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.launch(v, y)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / args.batch_reps
    y_eager = y.clone()
    t0 = time.perf_counter()
    b.capture(v, y)                     # the rounds the eager solve needed, plus a margin
    t_capture = time.perf_counter() - t0
    graph_rounds = b.graph_rounds
    b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / args.batch_reps
    same = bool(torch.equal(y, y_eager))
    s_graph, r_graph = b.results()
    # all rounds in one persistent (cooperative) launch, then as a replayed
    # graph of that launch
    y.zero_()
    b.launch_persistent(v, y)           # warm-up
    s_pers, r_pers = b.results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.launch_persistent(v, y)
    torch.cuda.synchronize()
    persistent = (time.perf_counter() - t0) / args.batch_reps
    pers_diff = float((y - y_eager).abs().max())
    b.capture_persistent(v, y)
    b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.replay()
    torch.cuda.synchronize()
    pers_graph = (time.perf_counter() - t0) / args.batch_reps
    b.results()
    # the same solve with one Newton product per round (eager)
    b1 = E.Batch(ns, ns, h, h, taus, bc="dirichlet0", tol=args.tol, dtype="f32")
    b1.set_pairs(False)
    b1.set_tiles(8, 8)
    b1.prepare()
    y1 = torch.zeros_like(v)
    b1.launch(v, y1)
    s1, r1 = b1.results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b1.launch(v, y1)
    torch.cuda.synchronize()
    single = (time.perf_counter() - t0) / args.batch_reps
    del b1, y1
    yy = y.cpu().numpy()
    errs = []
    for i, it in enumerate(inst):
        o, n2 = int(b.offsets[i]), it.n * it.n
        want = O.dirichlet_box_phi(1, (it.n, it.n), (h[i], h[i]), it.tau, v_host[o:o + n2])
        errs.append(float(np.linalg.norm(yy[o:o + n2] - want) / np.linalg.norm(want)))
    pts = int((ns * ns).sum())
    prods = sum(int(st["newton_steps"]) * it.n * it.n for st, it in zip(stats, inst))
    # per substep one first product (12 B per point: r read, w_1 and p
    # written) and pairs of products (16 B per point per pair); a product
    # taken alone past the degree bound is counted as half a pair
    newton_bytes = sum((12 * int(st["substeps"]) + 8 * (int(st["newton_steps"]) - int(st["substeps"])))
                       * it.n * it.n for st, it in zip(stats, inst))
    best = min(eager, graph, persistent, pers_graph)
    return {
        "workload": (f"{args.batch_count} independent 2D 5-point Dirichlet problems, sides "
                     f"log-uniform in [64, 1024], tau uniform in [1e-5, 1e-3], seed 0"),
        "value": pts / best,
        "unit": "grid-pts/s",
        "dtype": "f32 storage, f64 recurrences",
        "tol": args.tol,
        "total_points": pts,
        "eager_ms": 1e3 * eager,
        "graph_replay_ms": 1e3 * graph,
        "graph_rounds": graph_rounds,
        "persistent_ms": 1e3 * persistent,
        "persistent_graph_replay_ms": 1e3 * pers_graph,
        "persistent_rounds": r_pers,
        "persistent_max_abs_diff_vs_eager": pers_diff,
        "tiles": {"waves_march": tuned["tiles"], "chosen_by": "expi_batch_autotune",
                  "candidates_ms": tuned["candidates"]},
        "graph_capture_s": t_capture,
        "graph_equals_eager": same and r_graph == rounds,
        "rounds": rounds,
        "substeps_max": int(max(st["substeps"] for st in stats)),
        "newton_products": int(sum(st["newton_steps"] for st in stats)),
        "point_products_per_s": prods / best,
        "newton_gbs": newton_bytes / best / 1e9,
        "products_per_round": "two (pairs; the first product of a substep alone)",
        "single_products": {"eager_ms": 1e3 * single, "rounds": r1,
                            "newton_products": int(sum(st["newton_steps"] for st in s1)),
                            "tiles": [8, 8]},
        "err_vs_closed_form": {"max": max(errs), "median": float(np.median(errs)),
                               "worst_instance": int(np.argmax(errs))},
        "note": ("newton_gbs counts the Newton products' algorithmic bytes over the whole "
                 "solve time (start vectors, updates, stop tests and host gaps included): "
                 "per substep 12 B per point for the first product and 16 B per point for "
                 "each pair of products, FP32 vectors"),
    }


def run_csr(args):
    """The unstructured workload: phi_1(tau A) v for the negative graph
    Laplacian of a seeded random geometric graph in the unit cube, n = 2^20
    rows, about 27 stored entries per row (Morton-ordered points), int32
    indices, float64 values, tau rho(A) = 50, tol 1e-10, FP64.  Per-product
    algorithmic bytes: values and columns once (12 B per stored entry), row
    pointers (4 B per row), w read once, p read and written, w written
    (32 B per row)."""
    import torch
    import paper_1309_4616_amd as E
    import synth

    n = 1 << args.csr_log2n
    g = synth.rgg_negative_laplacian(n, seed=0)
    rho = synth.spectral_radius_symmetric(g)
    tau = 50.0 / rho
    op = E.CsrOp(g.n, g.rowptr, g.colind, g.val)
    v = torch.as_tensor(synth.uniform_vector(g.n, 0), device="cuda:0")
    y = torch.empty_like(v)
    params = E.LejaParams(profile=True)
    ws = op.workspace("f64")
    # lanes per row and waves per workgroup from the library's autotuner
    from paper_1309_4616_amd import autotune
    tuned = autotune.tune(op, "f64", reps=5, use_cache=False)
    E.phi_action(op, 1, tau, v, y=y, tol=1e-10, params=params, ws=ws)
    torch.cuda.synchronize()
    reps = args.csr_reps
    timed = 0
    ms = 0.0
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = E.phi_action(op, 1, tau, v, y=y, tol=1e-10, params=params, ws=ws)
        timed += st["timed_products"]
        ms += st["newton_ms"]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    per_product = 12 * g.nnz + 4 * (g.n + 1) + 32 * g.n
    avg_us = 1e3 * ms / max(timed, 1)
    gbs = per_product / (avg_us * 1e-6) / 1e9
    lanes = op.tiles()[0]
    traffic = counter_traffic(f"csr_sweep<1, double, double, {lanes}>") if args.csr_log2n == 20 else None
    return {
        "workload": (f"phi_1(tau A) v, A = negative graph Laplacian of a random geometric graph, "
                     f"n = 2^{args.csr_log2n}, {g.nnz / g.n:.1f} stored entries per row, "
                     f"tau rho(A) = 50, tol 1e-10, f64"),
        "value": g.n / wall,
        "unit": "rows/s (phi_1 results)",
        "ms_per_phi": 1e3 * wall,
        "substeps": st["substeps"],
        "newton_products": st["newton_steps"],
        "product_avg_us": avg_us,
        "product_gbs": gbs,
        "product_frac": gbs / HBM_PEAK_GBS,
        "algorithmic_bytes_per_product": per_product,
        "counted_bytes_per_product": traffic["bytes"] if traffic else None,
        "counted_bytes_source": traffic["profile"] if traffic else None,
        "lanes_per_row": lanes,
        "tiles": {"lanes_per_row_waves": tuned["tiles"][:2], "chosen_by": "expi_op_autotune",
                  "candidates_us": tuned["candidates"]},
        "nnz": int(g.nnz),
    }


def _time_launches(fn, reps: int) -> float:
    """Mean milliseconds per call of fn (launches on torch's current stream),
    timed with events around `reps` calls after two warm-up calls."""
    import torch
    for _ in range(2):
        fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / reps


def tuned_2d(E, op, dtype="f64"):
    """Autotune a 2D operator (single-product tiles, and the pair sweep's
    tile height against single products); returns what it chose."""
    from paper_1309_4616_amd import autotune
    res = autotune.tune(op, dtype, reps=5, use_cache=False)
    return {"tiles": list(op.tiles()), "single_us": res["us"], "pair_setting": op.pair_setting(),
            "pair_us_by_rows": {str(c[1]): round(t, 2) for c, t in res["candidates"] if c[0] == 0}}


def run_plain_2d(args):
    """The plain-method workload: phi_1(tau A) v for the 5-point Laplacian
    with homogeneous Dirichlet conditions on the 128 x 128 interior grid of
    the unit square (h = 1/129), v uniform in [-1, 1] (seeded), tau = 1e-4,
    tolerance 1e-10, FP64.  Wall time per call (inputs resident, the call's
    own status read-backs included) with 2D pair sweeps (the default) and
    with single products, and the average kernel time per launch from the
    library's profiling events; the operator is autotuned first (tiles, and
    the pair sweep's tile height).  Then the same at 8192^2, where the
    sweeps are bound by HBM, in FP64 and with FP32 storage."""
    import torch
    import paper_1309_4616_amd as E
    import synth

    n, tau, tol, reps = 128, 1e-4, 1e-10, args.plain_reps
    h = 1.0 / (n + 1)
    op = E.StencilOp((n, n), (h, h), "dirichlet0", coef=1.0)
    v = torch.as_tensor(synth.uniform_vector(n * n, 0), device="cuda:0")
    y = torch.empty_like(v)
    ws = op.workspace("f64")
    out = {"workload": "phi_1(tau A) v, 2D 5-point Dirichlet Laplacian, 128^2, h = 1/129, tau 1e-4, "
                       "tol 1e-10, FP64",
           "autotune": tuned_2d(E, op)}
    for key, pairs in (("pairs", True), ("singles", False)):
        params = E.LejaParams(pairs=pairs)
        for _ in range(10):
            E.phi_action(op, 1, tau, v, y=y, tol=tol, ws=ws, params=params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, st = E.phi_action(op, 1, tau, v, y=y, tol=tol, ws=ws, params=params)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        _, sp = E.phi_action(op, 1, tau, v, y=y, tol=tol, ws=ws, params=E.LejaParams(pairs=pairs, profile=True))
        rec = {"ms_per_call": ms, "degree": st["degree_last"], "substeps": st["substeps"],
               "matvecs": st["matvecs"], "pair_launches": st["pair_launches"],
               "single_launches": st["single_launches"]}
        if sp["timed_pairs"]:
            rec["pair_avg_us"] = 1e3 * sp["pair_ms"] / sp["timed_pairs"]
            # read w_j and p, write w_{j+2} and p: 32 B per point and launch
            rec["pair_gbs"] = 32.0 * n * n / (rec["pair_avg_us"] * 1e3)
        if sp["timed_products"]:
            rec["single_avg_us"] = 1e3 * sp["newton_ms"] / sp["timed_products"]
        out[key] = rec
    out["speedup_pairs"] = out["singles"]["ms_per_call"] / out["pairs"]["ms_per_call"]
    out["note"] = ("128 KiB per vector: every launch is latency bound (a few microseconds); pairs halve "
                   "the launches and the stop tests")
    del op, v, y, ws
    # the same operator on a grid whose sweeps are bound by HBM: 8192^2 (537 MB
    # per FP64 vector, as a 256^3 one), tau (b - a) = 30, tol 1e-8
    n = args.plain_large_n
    h = 1.0 / (n + 1)
    op = E.StencilOp((n, n), (h, h), "dirichlet0", coef=1.0)
    a, b = op.interval()
    tau = 30.0 / (b - a)
    v = torch.as_tensor(synth.uniform_vector(n * n, 1), device="cuda:0")
    y = torch.empty_like(v)
    for dt in ("f64", "f32"):
        bpp = 32.0 if dt == "f64" else 16.0   # read w_j, p; write w_{j+2}, p (or w_{j+1}, p)
        ws = op.workspace(dt)
        large = {"workload": f"phi_1(tau A) v, 2D 5-point Dirichlet Laplacian, {n}^2, tau (b - a) = 30, "
                             f"tol 1e-8, {'FP64' if dt == 'f64' else 'FP32 storage'}",
                 "autotune": tuned_2d(E, op, dt)}
        for key, pairs in (("pairs", True), ("singles", False)):
            params = E.LejaParams(pairs=pairs)
            E.phi_action(op, 1, tau, v, y=y, tol=1e-8, dtype=dt, ws=ws, params=params)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, st = E.phi_action(op, 1, tau, v, y=y, tol=1e-8, dtype=dt, ws=ws, params=params)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / 3
            _, sp = E.phi_action(op, 1, tau, v, y=y, tol=1e-8, dtype=dt, ws=ws,
                                 params=E.LejaParams(pairs=pairs, profile=True))
            rec = {"ms_per_call": ms, "degree": st["degree_last"], "pair_launches": st["pair_launches"],
                   "single_launches": st["single_launches"]}
            if sp["timed_pairs"]:
                us = 1e3 * sp["pair_ms"] / sp["timed_pairs"]
                rec.update(pair_avg_us=us, pair_gbs=bpp * n * n / (us * 1e3),
                           pair_frac=bpp * n * n / (us * 1e3) / HBM_PEAK_GBS)
            else:
                us = 1e3 * sp["newton_ms"] / sp["timed_products"]
                rec.update(single_avg_us=us, single_gbs=bpp * n * n / (us * 1e3),
                           single_frac=bpp * n * n / (us * 1e3) / HBM_PEAK_GBS)
            large[key] = rec
        large["speedup_pairs"] = large["singles"]["ms_per_call"] / large["pairs"]["ms_per_call"]
        large["note"] = (f"{bpp:.0f} B per point and launch for both: a pair sweep reads w_j, p and writes "
                         "w_{j+2}, p; a single product reads w_j, p and writes w_{j+1}, p")
        out["large" if dt == "f64" else "large_f32"] = large
        del ws
    del op, v, y
    torch.cuda.empty_cache()
    return out


def run_paper_tables(args):
    """The paper's single-kernel experiments on this GPU (context: the
    paper's numbers are on a Tesla C1060/C2075):
    - Table I: one 7-point product y = (alpha A + beta I) x at 256^3 and
      512^3, boundary handling none (interior only) or homogeneous Dirichlet,
      FP64 and FP32; and the two inhomogeneous Dirichlet data with the data
      evaluated inside the sweep or by a second kernel;
    - Table II: the product with c0 D(x, y) times the Laplacian,
      D = 1/sqrt(1 + x^2 + y^2) computed in the kernel;
    - Table III: the combustion nonlinearity over a vector, full precision
      and fast (hardware) exp, FP64 and FP32.
    Algorithmic traffic: one read and one write per point (16 B FP64, 8 B
    FP32); Gflop/s in the paper's convention of 10 flops per point."""
    import torch
    import paper_1309_4616_amd as E
    rows = []
    for n in args.table_sizes:
        pts = n ** 3
        h = (1.0 / (n + 1),) * 3
        for dt, td, bpp in (("f64", torch.float64, 16), ("f32", torch.float32, 8)):
            x = torch.rand(pts, dtype=td, device="cuda:0")
            y = torch.empty_like(x)
            # tile setting for this size and dtype from the library's autotuner
            # (it times the fused Newton sweep, the same traversal); every case
            # of the size uses it
            from paper_1309_4616_amd import autotune
            probe = E.StencilOp((n, n, n), h, "dirichlet0")
            tiles = autotune.tune(probe, dt, reps=3, use_cache=False)["tiles"]
            del probe
            torch.cuda.empty_cache()
            cases = [("I", "none (interior only)", E.StencilOp((n, n, n), h, "interior_only"), None),
                     ("I", "homogeneous Dirichlet", E.StencilOp((n, n, n), h, "dirichlet0"), None)]
            for kind in ("z1mz_xy", "sinpiz_expmxy"):
                for mode in ("in_kernel", "separate"):
                    op = E.StencilOp((n, n, n), h, "dirichlet0")
                    op.set_boundary_data(kind, mode)
                    cases.append(("I", f"Dirichlet data {kind}, {mode}", op, None))
            cases.append(("II", "D(x,y) Laplacian, D in kernel", E.StencilOp((n, n, n), h, "dirichlet0",
                                                                             coef=("dlap", 1.0)), None))
            for table, what, op, _ in cases:
                op.set_tiles(*tiles)
                ms = _time_launches(lambda: E.apply_op(op, 1.0, 0.5, x, y), args.table_reps)
                rows.append({"table": table, "n": n, "dtype": dt, "case": what, "ms": ms, "tiles": tiles,
                             "gbs": bpp * pts / (ms * 1e-3) / 1e9,
                             "gflops_10_per_point": 10 * pts / (ms * 1e-3) / 1e9})
            del x, y
            u = 1.0 + torch.rand(pts, dtype=td, device="cuda:0")
            g = torch.empty_like(u)
            for gk in ("combustion", "combustion_fast"):
                ms = _time_launches(lambda: E.nonlinearity(gk, u, g), args.table_reps)
                rows.append({"table": "III", "n": n, "dtype": dt, "case": gk, "ms": ms,
                             "gbs": bpp * pts / (ms * 1e-3) / 1e9})
            del u, g
            torch.cuda.empty_cache()
    return {"note": ("single launches timed with events on the stream, mean of "
                     f"{args.table_reps} after 2 warm-ups; gbs = one read + one write per point"),
            "rows": rows}


def run_combustion(args):
    """Table IV's workload: one exponential Euler step of the combustion model
    u' = Delta u + g(u), g(u) = (2 - u)/4 exp(20 (1 - 1/u)), on the 256^3
    interior grid with homogeneous Dirichlet boundaries (h = 1/257), u0 = 1,
    tau = 1e-4, tol = 1e-4 (the paper's settings), FP64 and FP32 storage,
    full and fast exp; and the second-order exponential Runge-Kutta step of
    the same problem."""
    import torch
    import paper_1309_4616_amd as E
    import synth
    n = 256
    op = E.StencilOp((n, n, n), (1.0 / (n + 1),) * 3, "dirichlet0")
    u0 = torch.as_tensor(synth.combustion_initial(n ** 3), device="cuda:0")
    out = {}
    for dt in ("f64", "f32"):
        for g in ("combustion", "combustion_fast"):
            u = u0.clone()
            E.expeuler_step(op, 1e-4, u, tol=1e-4, dtype=dt, g=g)     # warm-up
            reps = 5
            t = 0.0
            for _ in range(reps):
                u.copy_(u0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = E.expeuler_step(op, 1e-4, u, tol=1e-4, dtype=dt, g=g)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
            out[f"expeuler_{dt}_{g}"] = {"ms_per_step": 1e3 * t / reps, "matvecs": st["matvecs"],
                                         "substeps": st["substeps"], "degree": st["degree_last"]}
    u = u0.clone()
    E.exprk2_step(op, 1e-4, u, tol=1e-4, g="combustion")
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = E.exprk2_step(op, 1e-4, u, tol=1e-4, g="combustion")
    torch.cuda.synchronize()
    out["exprk2_f64_combustion"] = {"ms_per_step": 1e3 * (time.perf_counter() - t0),
                                    "matvecs": st["matvecs"]}
    out["paper_table_iv"] = ("40 products per step at tol 1e-4, 1.2 s (FP64) / 210 ms (FP32) on one "
                             "Tesla C2075; context only")
    return out


def run_spin_bath(args):
    """Sec. III-D's unstructured complex workload (Table V's shape): psi(t) =
    e^{-i t H} psi(0) for a Hermitian spin-bath matrix of `spin_spins` spins
    (2^spins rows, about 40 stored complex entries per row at 21 spins; the
    paper's Hamiltonian is not given, a synthetic one of the same shape
    stands in), t = 10, tol 1e-5, FP64, one call of expi_skew_phi_action.
    Per-product algorithmic bytes: values and columns once (20 B per stored
    entry), row pointers (4 B per row), w read once, p read and written, w
    written (64 B per row)."""
    import torch
    import paper_1309_4616_amd as E
    import synth
    t0 = time.perf_counter()
    g = synth.spin_bath_hamiltonian(args.spin_spins, seed=0)
    gen_s = time.perf_counter() - t0
    op = E.CsrComplexOp(g.n, g.rowptr, g.colind, g.val)
    del g.val
    # lanes per row and waves per workgroup from the library's autotuner
    from paper_1309_4616_amd import autotune
    tuned = autotune.tune(op, "f64", reps=3, use_cache=False)
    psi = torch.as_tensor(synth.complex_uniform_vector(g.n, 0), device="cuda:0")
    psi /= psi.norm()
    y = torch.empty_like(psi)
    ws = op.workspace("f64")
    params = E.LejaParams(profile=1)
    E.skew_phi_action(op, 0, args.spin_t, psi, y=y, tol=args.spin_tol, params=params, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = E.skew_phi_action(op, 0, args.spin_t, psi, y=y, tol=args.spin_tol, params=params, ws=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nnz = op.nnz
    per_product = 20 * nnz + 4 * (g.n + 1) + 64 * g.n
    avg_us = 1e3 * st["newton_ms"] / max(st["timed_products"], 1)
    lanes = tuned["tiles"][0]
    traffic = counter_traffic(f"csr_complex_sweep<1, {lanes}>") if args.spin_spins == 21 else None
    return {
        "workload": (f"e^(-i t H) psi, H Hermitian spin-bath matrix of {args.spin_spins} spins "
                     f"(n = 2^{args.spin_spins}, {nnz / g.n:.1f} complex entries per row), "
                     f"t = {args.spin_t:g}, tol {args.spin_tol:g}, f64"),
        "ms": 1e3 * wall,
        "substeps": st["substeps"],
        "products": st["matvecs"],
        "interval": [st["interval_a"], st["interval_b"]],
        "product_avg_us": avg_us,
        "product_gbs": per_product / (avg_us * 1e-6) / 1e9,
        "product_frac": per_product / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes_per_product": per_product,
        "counted_bytes_per_product": traffic["bytes"] if traffic else None,
        "counted_bytes_source": traffic["profile"] if traffic else None,
        "norm_drift": abs(y.norm().item() - 1.0),
        "tiles": {"lanes_per_row_waves": tuned["tiles"][:2], "chosen_by": "expi_op_autotune",
                  "candidates_us": tuned["candidates"]},
        "generate_s": gen_s,
        "paper_table_v": "21 spins to t = 10 at tol 1e-5: 7.7 s FP64 on one Tesla C2075 (its own Hamiltonian); context only",
    }


def gpu_states(args, dtype: str, steps: int):
    """The first `steps` exponential Euler steps of the benchmark workload
    from its u0 on the GPU (the timed configuration: pair sweeps, the given
    storage), states copied to the host after each step."""
    import torch
    import paper_1309_4616_amd as E
    import synth

    n = args.n
    h = 1.0 / n
    coef = synth.sine_coefficient(n, 0.5)
    op = E.StencilOp((n, n, n), (h, h, h), "neumann0",
                     coef=("separable", coef.c0, coef.c1, coef.tx, coef.ty, coef.tz))
    u = torch.as_tensor(synth.gaussian_bump_3d(n, seed=0), device="cuda:0")
    ws = op.workspace(dtype)
    out = []
    for _ in range(steps):
        E.expeuler_step(op, args.tau, u, tol=args.tol, dtype=dtype, ws=ws)
        out.append(u.cpu().numpy())
    del u, ws, op
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, gpu64, gpu32):
    """The oracle on a bounded sample of the same workload: the first
    `cpu_steps` exponential Euler steps of the 256^3 problem from the same
    u0 at the same tol, on one thread (scipy's sparse product is
    single-threaded; the BLAS pool is limited to one thread).  Operator
    assembly and the interval are not timed.  The GPU's states after the
    same steps (FP64 and FP32 storage) are compared with the oracle's, and
    one more oracle step at tol 1e-12 (untimed) gives the accuracy of the
    first step against a tighter reference."""
    import numpy as np
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import integrators as I
    from oracle import operators as O

    def relerr(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    n = args.n
    h = 1.0 / n
    with threadpool_limits(limits=1):
        time.sleep(0.5)   # BLAS threads used by earlier legs stop spinning
        A = O.stencil_matrix((n, n, n), (h, h, h), "neumann0",
                             coef=synth.sine_coefficient(n, 0.5).field())
        interval = O.gershgorin_interval(A)
        u0 = synth.gaussian_bump_3d(n, seed=0)
        u = u0
        states = []
        c0 = time.process_time()
        t0 = time.perf_counter()
        for _ in range(args.cpu_steps):
            u, st = I.expeuler_step(A, args.tau, u, args.tol, interval=interval)
            states.append(u)
        wall = time.perf_counter() - t0
        cpu = time.process_time() - c0
        ref, _ = I.expeuler_step(A, args.tau, u0, 1e-12, interval=interval)
    del A
    k = args.cpu_steps
    prev = states[-2] if k > 1 else u0
    errs = {
        "f64": {"state": relerr(gpu64[k - 1], states[-1]),
                "increment_last_step": relerr(gpu64[k - 1] - prev, states[-1] - prev),
                "first_step_increment_vs_tol_1e-12": relerr(gpu64[0] - u0, ref - u0)},
        "f32": {"state": relerr(gpu32[k - 1], states[-1]),
                "increment_last_step": relerr(gpu32[k - 1] - prev, states[-1] - prev),
                "first_step_increment_vs_tol_1e-12": relerr(gpu32[0] - u0, ref - u0)},
    }
    return {
        "value": n ** 3 * k / wall,
        "unit": "grid-pts/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"the first {k} exponential Euler steps of the same {n}^3 workload "
                   f"(tau={args.tau:g}, tol {args.tol:g}), float64 scipy.sparse on one thread "
                   f"of {cpu_model()} ({os.cpu_count()} logical CPUs on the host); "
                   f"operator assembly not timed; cpu/wall {cpu / wall:.2f}"),
        "wall_s": wall,
        "errors": errs,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # (about 30 ms of steps: the first tens of steps after start-up run
    # about 10% slower while the GPU clocks come up)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tau", type=float, default=1e-5)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-512", action="store_true", help="skip the FP32 512^3 leg")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--eval-steps", type=int, default=200)
    ap.add_argument("--sel-kappa", type=float, default=1.5,
                    help="weight of under-prediction in the selector's training loss")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-csr", action="store_true")
    ap.add_argument("--no-tables", action="store_true",
                    help="skip the paper's single-kernel experiments (Tables I-III)")
    ap.add_argument("--table-sizes", type=int, nargs="+", default=[256, 512])
    ap.add_argument("--table-reps", type=int, default=10)
    ap.add_argument("--no-combustion", action="store_true")
    ap.add_argument("--no-spin", action="store_true")
    ap.add_argument("--no-plain-2d", action="store_true")
    ap.add_argument("--plain-reps", type=int, default=200)
    ap.add_argument("--plain-large-n", type=int, default=8192)
    ap.add_argument("--spin-spins", type=int, default=21)
    ap.add_argument("--spin-t", type=float, default=10.0)
    ap.add_argument("--spin-tol", type=float, default=1e-5)
    ap.add_argument("--csr-only", action="store_true",
                    help="run only the CSR leg and print its JSON (for profiling)")
    ap.add_argument("--csr-log2n", type=int, default=20)
    ap.add_argument("--csr-reps", type=int, default=5)
    ap.add_argument("--no-pairs", action="store_true",
                    help="single Newton products only (no pair sweeps)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 512 MiB float64 tensor 3 times (a kernel of known "
                         "traffic, 512 MiB read + 512 MiB written per launch) to calibrate "
                         "hardware byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.csr_only:
        print("[bench] csr only", file=sys.stderr, flush=True)
        print(json.dumps({"csr": run_csr(args)}), flush=True)
        return
    # (not in counter runs: their only copies are the 512 MiB calibration)
    ceiling = None if args.copy_probe else copy_ceiling()
    if ceiling:
        print(f"[bench] device copy: {ceiling['2GiB']['gbs']:.0f} GB/s at 2 GiB, "
              f"{ceiling['256^3_f64']['gbs']:.0f} GB/s at 134 MB", file=sys.stderr, flush=True)
    print(f"[bench] f64: {args.warmup} warmup + {args.steps} timed steps at {args.n}^3", file=sys.stderr, flush=True)
    r64 = run_gpu(args, "f64")
    print(f"[bench] f64 done: {r64['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    r32 = None
    if not args.no_fp32:
        r32 = run_gpu(args, "f32")
        print(f"[bench] f32 done: {r32['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    r32_512 = None
    if not args.no_fp32 and not args.no_512:
        # FP32 storage beyond the 256 MB MALL: 512^3 (w, p 0.5 GB each), tau
        # scaled by (256/512)^2 to keep tau (b - a) and the degree of 256^3
        r32_512 = run_gpu(args, "f32", n=512, tau=args.tau * (args.n / 512.0) ** 2, steps=3, warmup=1)
        print(f"[bench] f32 512^3 done: {r32_512['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    learned = None
    if not args.no_learned:
        print(f"[bench] learned selector: log {args.train_steps} plain steps, train, "
              f"evaluate {args.eval_steps} held-out steps", file=sys.stderr, flush=True)
        learned = run_learned(args)
        print(f"[bench] learned done", file=sys.stderr, flush=True)
    batched = None
    if not args.no_batched:
        print(f"[bench] batched: {args.batch_count} problems, eager, graph and persistent",
              file=sys.stderr, flush=True)
        batched = run_batched(args)
        print(f"[bench] batched done: eager {batched['eager_ms']:.1f} ms, graph "
              f"{batched['graph_replay_ms']:.1f} ms, persistent {batched['persistent_ms']:.1f} ms "
              f"(graph {batched['persistent_graph_replay_ms']:.1f} ms)", file=sys.stderr, flush=True)
    csr = None
    if not args.no_csr:
        print("[bench] csr: random geometric graph Laplacian, n = 2^%d" % args.csr_log2n,
              file=sys.stderr, flush=True)
        csr = run_csr(args)
        print(f"[bench] csr done: {csr['product_avg_us']:.1f} us per product", file=sys.stderr, flush=True)
    tables = None
    if not args.no_tables:
        print("[bench] paper tables I-III: single products and the nonlinearity", file=sys.stderr, flush=True)
        tables = run_paper_tables(args)
        print("[bench] tables done", file=sys.stderr, flush=True)
    comb = None
    if not args.no_combustion:
        print("[bench] combustion step (Table IV workload)", file=sys.stderr, flush=True)
        comb = run_combustion(args)
        print("[bench] combustion done", file=sys.stderr, flush=True)
    spin = None
    if not args.no_spin:
        print(f"[bench] spin bath: {args.spin_spins} spins, e^(-i t H) psi", file=sys.stderr, flush=True)
        spin = run_spin_bath(args)
        print(f"[bench] spin bath done: {spin['ms']:.1f} ms, {spin['products']} products", file=sys.stderr,
              flush=True)
    plain2d = None
    if not args.no_plain_2d:
        print("[bench] plain method: phi_1 on the 128^2 Dirichlet Laplacian", file=sys.stderr, flush=True)
        plain2d = run_plain_2d(args)
        print(f"[bench] plain 2D done: {plain2d['pairs']['ms_per_call']:.3f} ms per call with pairs, "
              f"{plain2d['singles']['ms_per_call']:.3f} ms with singles; {args.plain_large_n}^2: "
              f"{plain2d['large']['pairs']['ms_per_call']:.2f} / {plain2d['large']['singles']['ms_per_call']:.2f} ms "
              f"(FP32 {plain2d['large_f32']['pairs']['ms_per_call']:.2f} / "
              f"{plain2d['large_f32']['singles']['ms_per_call']:.2f} ms)",
              file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] gpu states of the first {args.cpu_steps} steps (f64, f32)", file=sys.stderr, flush=True)
        g64 = gpu_states(args, "f64", args.cpu_steps)
        g32 = gpu_states(args, "f32", args.cpu_steps)
        print("[bench] cpu baseline (oracle, one thread) and errors vs the oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args, g64, g32)
        del g64, g32

    n = args.n
    alg = NEWTON_BYTES_PER_PT["f64"] * n ** 3
    if r64["pair_avg_us"]:
        # the dominant kernel: the pair sweep (two Newton products per launch;
        # algorithmic traffic read w_j and p, write w_{j+2} and p)
        traffic = counter_traffic("pair_sweep<1, 1, double, 0>") if n == 256 else None
        roofline = {
            "bound": "hbm",
            "kernel": "pair sweep: two fused Newton products per launch (3D separable stencil, f64)",
            "achieved": r64["pair_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": r64["pair_gbs"] / HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_unit": "HBM bytes per launch",
            "traffic_source": traffic["profile"] if traffic else None,
            "algorithmic_bytes_per_launch": alg,
            "bytes_per_point": NEWTON_BYTES_PER_PT["f64"],
            "products_per_launch": 2,
            "avg_launch_us": r64["pair_avg_us"],
            "launches_per_step": r64["pairs_per_step"],
            "single_product": {"avg_launch_us": r64["single_avg_us"], "achieved_gbs": r64["single_gbs"],
                               "launches_per_step": r64["singles_per_step"]},
            "autotune": r64["autotune"],
            "measured_copy_gbs": {k: v["gbs"] for k, v in ceiling.items()} if ceiling else None,
            "frac_of_copy_2GiB": r64["pair_gbs"] / ceiling["2GiB"]["gbs"] if ceiling else None,
        }
    else:
        traffic = counter_traffic("stencil_sweep<3, 1, 1, double, double, 2>") if n == 256 else None
        roofline = {
            "bound": "hbm",
            "kernel": "fused Newton product (3D separable-coefficient stencil, f64)",
            "achieved": r64["single_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": r64["single_gbs"] / HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_unit": "HBM bytes per launch",
            "traffic_source": traffic["profile"] if traffic else None,
            "algorithmic_bytes_per_launch": alg,
            "bytes_per_point": NEWTON_BYTES_PER_PT["f64"],
            "avg_launch_us": r64["single_avg_us"],
            "launches_per_step": r64["singles_per_step"],
        }
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "grid-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {
            "workload": f"expeuler-3d-reaction-diffusion-{n}^3",
            "grid": [n, n, n],
            "bc": "neumann0 (cell-centred, zero flux)",
            "coef": "a=1+0.5 sin(2pi x) sin(2pi y) sin(2pi z), separable tables",
            "nonlinearity": "u-u^3",
            "tau": args.tau,
            "tol": args.tol,
            "matvecs_per_step": r64["matvecs_per_step"],
            "newton_degrees": r64["degrees"],
            "point_products_per_s": r64["point_products_per_s"],
            "step_hbm_gbs": r64["step_gbs"],
        },
        "roofline": roofline,
        "cpu_baseline": ({k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")}
                         if cpu else None),
        "err_vs_oracle": (dict(cpu["errors"]["f64"], vs=(
            f"FP64 oracle, same u0 and tol, after {args.cpu_steps} steps; the last key: "
            f"step 1 against the oracle at tol 1e-12")) if cpu else None),
    }
    if r32:
        out["fp32_storage"] = {
            "value": r32["value"],
            "ms_per_step": r32["ms_per_step"],
            "matvecs_per_step": r32["matvecs_per_step"],
            "single_avg_us": r32["single_avg_us"],
            "single_gbs": r32["single_gbs"],
            "single_frac": (r32["single_gbs"] / HBM_PEAK_GBS) if r32["single_gbs"] else None,
            "pairs_per_step": r32["pairs_per_step"],
            "fused_starts_per_step": r32["fused_starts_per_step"],
            "step_hbm_gbs": r32["step_gbs"],
            "pair_avg_us": r32["pair_avg_us"],
            "pair_gbs": r32["pair_gbs"],
            "note": "w, p stored in float32; divided differences, norms, stop test and u in float64",
            "err_vs_oracle": cpu["errors"]["f32"] if cpu else None,
        }
    if r32_512:
        out["fp32_storage_512"] = {
            "workload": (f"the 3D workload at 512^3, tau {args.tau * (args.n / 512.0) ** 2:g} "
                         f"(tau (b - a) as at {args.n}^3), 3 steps, FP32 w and p"),
            "value": r32_512["value"],
            "ms_per_step": r32_512["ms_per_step"],
            "matvecs_per_step": r32_512["matvecs_per_step"],
            "pairs_per_step": r32_512["pairs_per_step"],
            "pair_avg_us": r32_512["pair_avg_us"],
            "pair_gbs": r32_512["pair_gbs"],
            "pair_frac": (r32_512["pair_gbs"] / HBM_PEAK_GBS) if r32_512["pair_gbs"] else None,
            "single_avg_us": r32_512["single_avg_us"],
            "single_gbs": r32_512["single_gbs"],
            "note": ("working set 3 x 0.54 GB, beyond the MALL; pair sweeps with four waves per "
                     "row and two output rows per workgroup (16 B per point and launch: read w, p; "
                     "write w'', p)"),
        }
    if learned:
        out["learned_vs_plain"] = learned
    if batched:
        out["batched"] = batched
    if csr:
        out["csr"] = csr
    if tables:
        out["paper_tables"] = tables
    if comb:
        out["combustion"] = comb
    if spin:
        out["spin_bath"] = spin
    if plain2d:
        out["plain_2d"] = plain2d
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
