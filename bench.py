"""Benchmark of the nonlocal-operator hot path on one MI355X.

Headline (one "step" = one application of L_delta to the 2D workload):
  2D nonlocal diffusion, 1024^2 grid, variable horizon
  delta(x) = 4h (1 + 0.5 sin 2 pi x1 cos 2 pi x2) (m in [2, 6]), lognormal c(x),
  fractional profile r^-(2+2s) with s = 1/2 (discrete normalisation), u a seeded
  Gaussian random field, FP32 storage with compensated sums, direct quadrature.

The JSON line also carries the other rows of the hot path (FP64, the Section 3
hierarchical evaluation, peridynamics, the batched CG solve and the learned
preconditioner when built) under "rows".  Inputs are resident in HBM before
timing starts; plan set-up is excluded (it is the amortised initialisation).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, warmup):
    """Run fn() warmup times, then time exactly `steps` calls with events on the
    current stream (the stream the library launches on)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def timed_graph(fn, steps, warmup):
    """Like timed(), with the launches replayed from a HIP graph: G calls of fn
    are captured once (G the largest divisor of steps up to 100) and the graph
    is replayed steps / G times between the events, so host-side call overhead
    does not starve the GPU.  The output of a replay is checked against an
    eager call first."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    g_n = max(d for d in range(1, min(steps, 100) + 1) if steps % d == 0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(g_n):
            fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps // g_n):
        graph.replay()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def src_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1905_08375_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(tag, kernel_src, variant=None):
    """HBM traffic per launch measured with rocprofv3 counters (profiles/), or None
    when the kernel source changed since the counters were taken or the timed
    launch used another tile variant than the measured one."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("src_hash") != src_hash(*kernel_src):
        return None
    if variant is not None and rec.get("variant", variant) != variant:
        return None
    return rec.get("bytes_per_launch")


def J_of(info):
    """Half-width of the compile-time offset table: (J + 1)^2 - 1 >= k_max."""
    J = 1
    while (J + 1) ** 2 - 1 < info.k_max:
        J += 1
    return J


def c2_inputs(prec):
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    n, R = 1024, 6
    w = F.diffusion_2d(n=n)
    npt = np.float64 if prec == ndl.NDL_F64 else np.float32  # F32C and F32K store FP32
    d = torch.from_numpy(w["delta"].astype(npt)).cuda()
    c = torch.from_numpy(w["coef"].astype(npt)).cuda()
    u = torch.from_numpy(F.pad(w["u"], R).astype(npt)).cuda()
    return w, n, R, d, c, u


def bench_apply(prec, fast, steps, warmup, variant=None):
    import torch
    from paper_1905_08375_amd import ndl
    w, n, R, d, c, u = c2_inputs(prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, prec=prec), want_fast=fast, keep=(d, c))
    if fast:
        ndl.ndl_autotune(plan)  # plan-time choice of the hierarchical method (dyadic panels or rows)
    elif variant is None:
        ndl.ndl_autotune(plan)  # plan-time tile choice (excluded from timing)
    else:
        ndl.ndl_plan_set_variant(plan, variant)  # a fixed tile (profiling runs)
    out = torch.empty((n, n), dtype=u.dtype, device="cuda")
    fn = (lambda: ndl.ndl_apply_fast(plan, u, out, 1)) if fast else (lambda: ndl.ndl_apply(plan, u, out, 1))
    fn()
    eager = out.clone()
    secs, wall = timed_graph(fn, steps, warmup)
    if not torch.equal(out, eager):
        raise RuntimeError("graph replay of the apply differs from the eager call")
    info = plan.info()
    plan.close()
    return dict(seconds=secs, wall=wall, n_points=n * n, info=info, out=out)


def bench_solve(count=64, rtol=1e-8, prec=None, max_iter=None):
    """64 batched case (b) solves on uneven grids {256..1024}^2, m in [2, 8]."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    prec = ndl.NDL_F32C if prec is None else prec
    npt = np.float64 if prec == ndl.NDL_F64 else np.float32
    sizes = F.solve_sizes(count)
    plans, bs, xs = [], [], []
    R = 8
    for i, n in enumerate(sizes):
        w = F.solve_instance_2d(n, i)
        d = torch.from_numpy(w["delta"].astype(npt)).cuda()
        c = torch.from_numpy(w["coef"].astype(npt)).cuda()
        plans.append(ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, form=ndl.NDL_DIV, prec=prec), keep=(d, c)))
        bs.append(torch.from_numpy(w["b"]).cuda())
        xs.append(torch.zeros((n, n), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, reps = ndl.ndl_cg_solve(plans, bs, xs, rtol=rtol, max_iter=max_iter or 200000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pts = sum(n * n for n in sizes)
    return {"seconds_to_1e-8": el, "problems": count, "points": pts, "rc": rc,
            "max_rel_res_fp64": max(r.rel_res_fp64 for r in reps), "all_converged": all(r.converged for r in reps),
            "max_iters": max(r.iters for r in reps), "outer_steps": max(r.outer for r in reps),
            "precision": "fp32 inner (compensated apply), fp64 reductions and refinement"}


def bench_pcg_3d(n=256, seed=100, train_steps=0, max_iter=None):
    """3D 256^3 case (b) solve to 1e-8: plain Jacobi-CG vs the learned two-level
    preconditioner (weights from precond_train.WEIGHTS when present, else the
    network is trained here on full fields for `train_steps` steps; training
    time is reported separately and is not part of the solve times)."""
    from paper_1905_08375_amd import ndl
    from paper_1905_08375_amd import precond_train as PT
    source = "untrained (output layer at zero: plain Jacobi)"
    train_s = 0.0
    if os.path.exists(PT.WEIGHTS):
        net = PT.load_net(PT.WEIGHTS)
        source = os.path.relpath(PT.WEIGHTS, ROOT) + " (linear mode)"
    else:
        net = PT.new_net(seed=1)
        if train_steps > 0:
            t0 = time.perf_counter()
            data = PT.make_pairs(n, range(2), ks=PT.TRAIN_KS, log=log)
            PT.train(net, data, steps=train_steps, log=log)
            train_s = time.perf_counter() - t0
            source = f"trained here ({train_steps} steps, linear mode)"
    res = PT.compare(net, n=n, seed=seed, max_iter=max_iter)
    res["weights"] = source
    res["training_seconds"] = train_s
    return res


def bench_net(n=256, seed=100, reps=50):
    """One inference of the shipped preconditioner network (linear mode) on a
    256^3 residual through ndl_precond_apply: input scaling, 13 BF16 MFMA
    convolutions, 3 poolings, the output unscaling; ms per inference."""
    import torch
    from paper_1905_08375_amd import ndl
    from paper_1905_08375_amd import precond_train as PT
    if not os.path.exists(PT.WEIGHTS):
        return {"skipped": "no trained weights in the tree"}
    net = PT.load_net(PT.WEIGHTS)
    plan, b, _, _ = PT.problem_3d(n, seed)
    g = torch.Generator(device="cuda").manual_seed(seed)
    r = torch.randn((n, n, n), device="cuda", generator=g)
    z = torch.empty_like(r)
    for _ in range(3):
        ndl.ndl_precond_apply(net, plan, r, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ndl.ndl_precond_apply(net, plan, r, z)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    plan.close()
    return {"ms_per_inference": ms, "voxels": n ** 3, "layers": 13, "precision": "bf16 activations and weights, fp32 accumulation"}


def bench_sweep(n=1024, ms=(2, 4, 8, 16, 32, 64), example1=True):
    """Direct sum vs the Section 3 evaluation for the constant profile (p^0 = g
    exactly, so the hierarchical path is pure panel sums) at growing horizon
    m = delta n, by the dyadic panels (fast_ms) and by the row prefix sums
    (rows_ms); the last point is the paper's Example 1 (delta = 1/2, direct
    sum out of reach of the LDS tile, hierarchical only)."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    prec = ndl.NDL_F32C
    out = []
    cases = [(m, m / n) for m in ms] + ([(n // 2, 0.5)] if example1 else [])
    u_base = F.grf(n, 2, 1.0, 0.1, 6, 1)
    c = torch.from_numpy(np.exp(F.grf(n, 2, 0.5, 0.1, 6, 2)).astype(np.float32)).cuda()
    for m, delta in cases:
        R = int(np.ceil(m)) + 1
        d = torch.full((n, n), delta, dtype=torch.float32, device="cuda")
        u = torch.from_numpy(F.pad(u_base, R).astype(np.float32)).cuda()  # zero collar
        plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, kernel=ndl.NDL_G_CONST, prec=prec), want_fast=1,
                                   keep=(d, c))
        o = torch.empty((n, n), dtype=torch.float32, device="cuda")
        row = {"m": m, "neighbours_per_node": plan.info().pairs_per_point}

        def run(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            k = int(max(2, min(50, 0.25 / max(first, 1e-6))))
            secs, _ = timed(fn, k, 1)
            return secs / k

        row["fast_ms"] = run(lambda: ndl.ndl_apply_fast(plan, u, o, 1)) * 1e3
        ndl.ndl_plan_set_fast_method(plan, 1)  # the row variant of Steps 2 and 3
        row["rows_ms"] = run(lambda: ndl.ndl_apply_fast(plan, u, o, 1)) * 1e3
        ndl.ndl_plan_set_fast_method(plan, 0)
        if delta < 0.5:
            ndl.ndl_autotune(plan)
            row["direct_ms"] = run(lambda: ndl.ndl_apply(plan, u, o, 1)) * 1e3
            row["direct_tile"] = [plan.info().tile_x, plan.info().tile_y]
            row["fast_speedup"] = row["direct_ms"] / row["fast_ms"]
            row["rows_speedup"] = row["direct_ms"] / row["rows_ms"]
        plan.close()
        out.append(row)
    return {"n": n, "profile": "const (p^0 exact)", "precision": "fp32 data, fp64 panel sums", "points": out}


def bench_pd(steps=5, batch=8, n=2048, fast=False):
    """Peridynamics on 8 fields of 2048^2 (m in [3, 12], Voronoi c, rotation plus
    a random field): the direct sum (FP32, Kahan), or the hierarchical path
    (degree-2 panel moments per component, F32C) with fast=True."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    R = 12
    w = F.peridynamic_2d(n=n, batch=batch, R=R)
    d = torch.from_numpy(w["delta"].astype(np.float32)).cuda()
    c = torch.from_numpy(w["coef"].astype(np.float32)).cuda()
    u = torch.from_numpy(w["u"].astype(np.float32)).cuda()
    prec = ndl.NDL_F32C if fast else ndl.NDL_F32K
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_INV_R,
                                                prec=prec), want_fast=int(fast), keep=(d, c))
    if not fast:
        ndl.ndl_autotune_apply(plan, u, batch)  # tile tuned on these fields at this batch (plan time)
    out = torch.empty((batch, 2, n, n), dtype=torch.float32, device="cuda")
    fn = (lambda: ndl.ndl_apply_fast(plan, u, out, batch)) if fast else (lambda: ndl.ndl_apply(plan, u, out, batch))
    secs, _ = timed(fn, steps, 1)
    per = secs / steps
    inf = plan.info()
    res = {"ms_per_batch_apply": per * 1e3, "gpoint_fields_per_s": batch * n * n / per / 1e9,
           "pairs_per_point": inf.pairs_per_point}
    if fast:
        res["levels"] = inf.fast_levels
    else:
        res["tile"] = [inf.tile_x, inf.tile_y]
    plan.close()
    return res


def bench_sym(n=1024, steps=400, cg_n=256):
    """The kernel-averaged symmetric form omega_s = (omega_x(y) + omega_y(x))/2
    on the 1024^2 workload (FP32 with Kahan sums, r^-3 profile): the direct sum
    and the fast evaluation (hierarchical gather plus its adjoint scatter), ms
    per apply from graph replays; and Jacobi-CG to 1e-8 in FP64 through the
    direct apply on the same recipe at 256^2."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    R = 6
    w = F.diffusion_2d(n=n)
    d = torch.from_numpy(w["delta"].astype(np.float32)).cuda()
    c = torch.from_numpy(w["coef"].astype(np.float32)).cuda()
    u = torch.from_numpy(F.pad(w["u"], R).astype(np.float32)).cuda()
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    res = {"n": n, "profile": "r^-3 (s = 1/2)", "precision": "fp32 storage, fp32 Kahan sums"}
    for fast in (False, True):
        plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, form=ndl.NDL_SYM, prec=ndl.NDL_F32K),
                                   want_fast=int(fast), keep=(d, c))
        fn = (lambda: ndl.ndl_apply_fast(plan, u, out, 1)) if fast else (lambda: ndl.ndl_apply(plan, u, out, 1))
        secs, _ = timed_graph(fn, steps, 20)
        res["fast_ms" if fast else "direct_ms"] = secs / steps * 1e3
        plan.close()
    w = F.diffusion_2d(n=cg_n)
    d = torch.from_numpy(w["delta"]).cuda()
    c = torch.from_numpy(w["coef"]).cuda()
    b = torch.from_numpy(np.random.default_rng(cg_n).standard_normal((cg_n, cg_n))).cuda()
    x = torch.zeros_like(b)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, cg_n, R, d, c, form=ndl.NDL_SYM, prec=ndl.NDL_F64), keep=(d, c))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, reps = ndl.ndl_cg_solve([plan], [b], [x], rtol=1e-8)
    torch.cuda.synchronize()
    res["cg_256_fp64"] = {"seconds": time.perf_counter() - t0, "iters": reps[0].iters, "rc": rc,
                          "rel_res": reps[0].rel_res_fp64}
    plan.close()
    return res


def bench_pd3d(n=128, steps=20):
    """3D linear bond-based peridynamics on one 128^3 displacement field (3
    components; m(x) = 3 + sin sin sin in [2, 4], lognormal c, GRF
    displacements): the direct sum with the 1/r and the conical (1 - r)/r
    micromoduli (FP32, Kahan sums), and the hierarchical path with the 1/r
    profile (FP32 data, FP64 moments); ms per apply."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    R = 5
    w = F.diffusion_3d(n=n)
    d = torch.from_numpy(w["delta"].astype(np.float32)).cuda()
    c = torch.from_numpy(w["coef"].astype(np.float32)).cuda()
    uu = np.stack([F.pad(1e-3 * F.grf(n, 3, 1.0, 0.1, 5, 300 + k), R) for k in range(3)])
    u = torch.from_numpy(uu.astype(np.float32)).cuda()
    out = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
    res = {"n": n, "components": 3}
    for nm, kernel, prec, fast in [("direct_inv_r_ms", ndl.NDL_G_INV_R, ndl.NDL_F32K, False),
                                   ("direct_cone_ms", ndl.NDL_G_CONE, ndl.NDL_F32K, False),
                                   ("fast_inv_r_ms", ndl.NDL_G_INV_R, ndl.NDL_F32C, True)]:
        plan = ndl.ndl_plan_create(ndl.make_problem(3, n, R, d, c, model=ndl.NDL_PERIDYNAMIC, kernel=kernel,
                                                    prec=prec), want_fast=int(fast), keep=(d, c))
        fn = (lambda: ndl.ndl_apply_fast(plan, u, out, 1)) if fast else (lambda: ndl.ndl_apply(plan, u, out, 1))
        secs, _ = timed(fn, steps, 2)
        res[nm] = secs / steps * 1e3
        res["pairs_per_point"] = plan.info().pairs_per_point
        plan.close()
    return res


def bench_example2(sizes=(4096, 8192, 16384)):
    """The paper's second example at growing N: 1D, delta(x) = (1/4)(1 +
    exp(-20 (x - 1/2)^2)) (N/4 to N/2 neighbours per side), the K = 3
    polynomial p^6, zero volume constraint, FP64; the hierarchical path (panel
    moments of degree 6) against the direct sum."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    p6 = (35 / 16, -35 / 16, 21 / 16, -5 / 16)
    pts = []
    for N in sizes:
        delta = F.example2_delta(N)
        R = int(np.ceil(delta.max() * N)) + 1
        d = torch.from_numpy(delta).cuda()
        c = torch.ones(N, dtype=torch.float64, device="cuda")
        g = np.random.default_rng(N)
        u = torch.zeros(N + 2 * R, dtype=torch.float64, device="cuda")
        u[R:R + N] = torch.from_numpy(g.standard_normal(N)).cuda()
        plan = ndl.ndl_plan_create(ndl.make_problem(1, N, R, d, c, kernel=ndl.NDL_G_POLY, poly=p6,
                                                    norm=ndl.NDL_NORM_NONE, prec=ndl.NDL_F64), want_fast=1,
                                   keep=(d, c))
        o = torch.empty(N, dtype=torch.float64, device="cuda")
        row = {"N": N, "neighbours_per_node": plan.info().pairs_per_point}
        for nm, fn in [("fast_ms", lambda: ndl.ndl_apply_fast(plan, u, o, 1)),
                       ("direct_ms", lambda: ndl.ndl_apply(plan, u, o, 1))]:
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            k = int(max(2, min(50, 0.25 / max(first, 1e-6))))
            secs, _ = timed(fn, k, 1)
            row[nm] = secs / k * 1e3
        row["fast_speedup"] = row["direct_ms"] / row["fast_ms"]
        plan.close()
        pts.append(row)
    return {"profile": "p^6 (K = 3)", "precision": "fp64", "points": pts}


def bench_big(steps=200, n=4096):
    """The headline kernel on a 4096^2 grid with the same horizon and
    coefficient recipe (m in [2, 6]): launch latency amortised over 16x the
    nodes."""
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    R = 6
    w = F.diffusion_2d(n=n)
    d = torch.from_numpy(w["delta"].astype(np.float32)).cuda()
    c = torch.from_numpy(w["coef"].astype(np.float32)).cuda()
    u = torch.from_numpy(F.pad(w["u"], R).astype(np.float32)).cuda()
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, prec=ndl.NDL_F32K), keep=(d, c))
    ndl.ndl_autotune(plan)
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    secs, _ = timed_graph(lambda: ndl.ndl_apply(plan, u, out, 1), steps, 10)
    per = secs / steps
    inf = plan.info()
    plan.close()
    return {"n": n, "us_per_apply": per * 1e6, "gpoint_per_s": n * n / per / 1e9,
            "hbm_frac": 16.0 * n * n / per / 1e9 / HBM_PEAK_GBS, "tile": [inf.tile_x, inf.tile_y]}


def bench_1d(steps=200):
    import torch
    from paper_1905_08375_amd import fields as F
    from paper_1905_08375_amd import ndl
    d1 = F.diffusion_1d()
    n, R = 4096, 41
    dd = torch.from_numpy(d1["delta"]).cuda()
    cc = torch.from_numpy(d1["coef"]).cuda()
    u = torch.from_numpy(F.pad(d1["u"], R)).cuda()
    plan = ndl.ndl_plan_create(ndl.make_problem(1, n, R, dd, cc, kernel=ndl.NDL_G_CONST,
                                                norm=ndl.NDL_NORM_CONTINUOUS, prec=ndl.NDL_F64), keep=(dd, cc))
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    secs, _ = timed_graph(lambda: ndl.ndl_apply(plan, u, out, 1), steps, 10)
    # the same field through case (b) (per-pair cutoff and coefficient)
    plan_b = ndl.ndl_plan_create(ndl.make_problem(1, n, R, dd, cc, form=ndl.NDL_DIV, kernel=ndl.NDL_G_CONST,
                                                  norm=ndl.NDL_NORM_CONTINUOUS, prec=ndl.NDL_F64), keep=(dd, cc))
    secs_b, _ = timed_graph(lambda: ndl.ndl_apply(plan_b, u, out, 1), steps, 10)
    return {"us_per_apply": secs / steps * 1e6, "case_b_us_per_apply": secs_b / steps * 1e6,
            "note": "4096 nodes, graph replays: launch-latency bound"}


def calib_copy(mib=256, reps=20):
    """A plain copy of known size (256 MiB read + 256 MiB written per copy), the
    reference that scales the rocprofv3 FETCH_SIZE / WRITE_SIZE counters of the
    measured kernels to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"mib": mib, "copies": reps}


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle on the same workload (FP32-rounded inputs), on the host cores."""
    import oracle as O
    from paper_1905_08375_amd import fields as F
    n, R = 1024, 6
    w = F.diffusion_2d(n=n)
    P = O.Problem(dim=2, n=n, R=R, kernel="frac", s=0.5)
    d = w["delta"].astype(np.float32).astype(np.float64)
    c = w["coef"].astype(np.float32).astype(np.float64)
    u = F.pad(w["u"], R).astype(np.float32).astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    while True:
        O.apply(P, d, c, u)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 50:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    return {"value": reps * n * n / el / 1e9, "unit": "Gpoint-applies/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} full applies of the 1024^2 workload (FP64 direct sum, OpenMP over nodes), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-rows", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="run one row only (profiling): cg64, pcg3d, net, pd, pdfast, pd3d, sym, ex2, big, sweep, fast, f64, 1d, "
                         "or calib (the counter calibration copy)")
    ap.add_argument("--cg-iters", type=int, default=0, help="cap the solver iterations (profiling)")
    ap.add_argument("--variant", type=int, default=None,
                    help="fixed tile variant for the headline (and --only f64) instead of the autotuner's "
                         "(profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1905_08375_amd import ndl
    assert torch.cuda.is_available(), "needs a GPU"
    ndl.lib()
    if args.only:
        fn = {"cg64": lambda: bench_solve(max_iter=args.cg_iters or None),
              "pcg3d": lambda: bench_pcg_3d(max_iter=args.cg_iters or None),
              "net": bench_net, "pd": bench_pd, "pdfast": lambda: bench_pd(fast=True), "ex2": bench_example2,
              "big": bench_big, "1d": bench_1d, "calib": calib_copy, "sweep": bench_sweep, "f64": lambda: bench_apply(ndl.NDL_F64, False, args.steps, args.warmup, args.variant)["seconds"],
              "fast": lambda: bench_apply(ndl.NDL_F32C, True, args.steps, args.warmup)["seconds"],
              "sym": bench_sym, "pd3d": bench_pd3d}[args.only]
        print(json.dumps({"only": args.only, "result": fn()}, default=str), flush=True)
        return

    log("headline: 2D 1024^2 direct apply, FP32 with Kahan-compensated sums")
    head = bench_apply(ndl.NDL_F32K, False, args.steps, args.warmup, args.variant)
    N = head["n_points"]
    per = head["seconds"] / args.steps
    value = N * args.steps / head["seconds"] / 1e9
    alg_bytes = 16.0 * N  # u, k_i, s_i read once, Lu written once, 4 B each
    traffic = load_traffic("c2_direct_f32k", ["direct2d.inc"], int(head["info"].variant))
    roof = {"bound": "hbm", "achieved": alg_bytes / per / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg_bytes / per / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_nd2<float,J=%d,E=-3,PY,NW,MODE=2,%s> tile %dx%d (FP32, Kahan)" % (
                J_of(head["info"]), "column order" if head["info"].pair_order else "sorted pairs",
                head["info"].tile_x, head["info"].tile_y), "alg_bytes_per_launch": alg_bytes}
    rows = {}
    if not args.no_rows:
        k = max(50, args.steps // 4)
        log("row: FP64 direct")
        r = bench_apply(ndl.NDL_F64, False, k, 20)
        rows["direct_f64"] = {"gpoint_per_s": N * k / r["seconds"] / 1e9, "us_per_apply": r["seconds"] / k * 1e6,
                              "hbm_frac": 28.0 * N / (r["seconds"] / k) / 1e9 / HBM_PEAK_GBS,
                              "tile": [r["info"].tile_x, r["info"].tile_y]}
        log("row: FP32 storage, FP64-carried sums")
        r = bench_apply(ndl.NDL_F32C, False, k, 20)
        rows["direct_f32c"] = {"gpoint_per_s": N * k / r["seconds"] / 1e9, "us_per_apply": r["seconds"] / k * 1e6,
                               "hbm_frac": 16.0 * N / (r["seconds"] / k) / 1e9 / HBM_PEAK_GBS,
                               "tile": [r["info"].tile_x, r["info"].tile_y]}
        for prec, nm in [(ndl.NDL_F32C, "fast_f32c"), (ndl.NDL_F64, "fast_f64")]:
            log("row:", nm)
            r = bench_apply(prec, True, k, 20)
            rows[nm] = {"gpoint_per_s": N * k / r["seconds"] / 1e9, "us_per_apply": r["seconds"] / k * 1e6,
                        "method": "rows" if r["info"].fast_method == 1 else "dyadic panels"}
        log("row: direct vs hierarchical sweep over the horizon (constant profile)")
        rows["sweep_const_2d_1024"] = bench_sweep()
        log("row: 1D 4096 direct FP64")
        rows["direct_1d_4096_f64"] = bench_1d()
        log("row: direct apply at 4096^2")
        rows["direct_f32k_4096"] = bench_big()
        log("row: peridynamics 2048^2 x 8 fields")
        rows["pd_2048x8_f32k"] = bench_pd()
        log("row: peridynamics 2048^2 x 8 fields, hierarchical")
        rows["pd_2048x8_fast_f32c"] = bench_pd(fast=True)
        log("row: 3D peridynamics 128^3, 1/r and conical micromoduli")
        rows["pd_3d_128"] = bench_pd3d()
        log("row: kernel-averaged symmetric form, 1024^2")
        rows["sym_2d_1024"] = bench_sym()
        log("row: the paper's second example (1D, K = 3) at growing N")
        rows["example2_1d_k3"] = bench_example2()
        log("row: 64 batched solves to 1e-8")
        rows["cg_64_uneven_to_1e-8"] = bench_solve()
        log("row: 3D 256^3 PCG to 1e-8, plain vs learned")
        rows["pcg_3d_256_to_1e-8"] = bench_pcg_3d()
        log("row: preconditioner network inference at 256^3")
        rows["precond_net_3d_256"] = bench_net()
    cpu = None if args.no_cpu else cpu_baseline()
    line = {
        "metric": "Gpoint-applies/s of L_delta (2D var. horizon); PCG time to 1e-8: learned vs plain",
        "value": value,
        "unit": "Gpoint-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2d-nonlocal-diffusion-1024x1024-variable-horizon-m2to6-frac-s0.5-direct",
                   "n": 1024, "collar": 6, "k_max": int(head["info"].k_max), "k_min": int(head["info"].k_min),
                   "precision": "fp32-storage-fp32-kahan-sums", "parallelism": "single-gpu",
                   "tile": [int(head["info"].tile_x), int(head["info"].tile_y)],
                   "tile_variant": int(head["info"].variant)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
