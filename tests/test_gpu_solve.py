"""Batched CG (ndl_cg_solve) against the FP64 oracle: -L_div x = b to a relative
FP64 true residual of 1e-8, several uneven problems in one call."""
import numpy as np
import pytest

import oracle as O
from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import dev, rel_l2, say

pytestmark = pytest.mark.gpu


def problems(sizes, dim=2, seed=0, mlo=2.0, mhi=8.0):
    out = []
    for i, n in enumerate(sizes):
        g = np.random.default_rng(seed + i)
        X = F.mesh(n, dim)
        ph = g.uniform(0, 1, size=2)
        m = (mlo + mhi) / 2 + (mhi - mlo) / 2 * np.sin(2 * np.pi * (X[0] + ph[0])) * np.cos(2 * np.pi * (X[-1] + ph[1]))
        c = np.exp(F.grf(n, dim, 0.5, 0.1, 4, 2000 + seed + i))
        b = g.standard_normal((n,) * dim)
        out.append((n, m / n, c, b))
    return out


def run(probs, prec, dim=2, R=8, **kw):
    import torch
    plans, bs, xs, keep = [], [], [], []
    for n, delta, c, b in probs:
        d_d, d_c = dev(delta, prec), dev(c, prec)
        plans.append(ndl.ndl_plan_create(ndl.make_problem(dim, n, R, d_d, d_c, form=ndl.NDL_DIV, prec=prec),
                                         keep=(d_d, d_c)))
        bs.append(torch.from_numpy(b.astype(np.float64)).cuda())
        xs.append(torch.zeros((n,) * dim, dtype=torch.float64, device="cuda"))
    rc, reps = ndl.ndl_cg_solve(plans, bs, xs, **kw)
    torch.cuda.synchronize()
    return rc, reps, [x.cpu().numpy() for x in xs]


def oracle_relres(n, delta, c, b, x, prec, dim=2, R=8):
    P = O.Problem(dim=dim, n=n, R=R, form="div", kernel="frac")
    npt = np.float64 if prec == ndl.NDL_F64 else np.float32
    d64 = delta.astype(npt).astype(np.float64)
    c64 = c.astype(npt).astype(np.float64)
    Ax = -O.apply(P, d64, c64, F.pad(x, R))
    return np.linalg.norm(b - Ax) / np.linalg.norm(b), d64, c64


@pytest.mark.parametrize("prec", [ndl.NDL_F64, ndl.NDL_F32C])
def test_batched_cg_reaches_1e8(prec):
    say(f"case cg prec={prec}")
    probs = problems([40, 56, 64, 33])
    rc, reps, xs = run(probs, prec, rtol=1e-8)
    assert rc == ndl.NDL_OK, ndl.ndl_last_error()
    for (n, delta, c, b), rep, x in zip(probs, reps, xs):
        rr, d64, c64 = oracle_relres(n, delta, c, b, x, prec)
        say(f"  n={n} iters={rep.iters} outer={rep.outer} gpu_res={rep.rel_res_fp64:.2e} oracle_res={rr:.2e}")
        assert rep.converged == 1
        assert rep.rel_res_fp64 <= 1e-8
        assert rr <= 1.05e-8
        # the oracle's own solve: x agrees within the residual-implied bound
        P = O.Problem(dim=2, n=n, R=8, form="div", kernel="frac")
        xo, it, rro, ok = O.cg_div(P, d64, c64, b, rtol=1e-10)
        assert ok
        assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)
        if prec == ndl.NDL_F64:
            _, it8, _, _ = O.cg_div(P, d64, c64, b, rtol=1e-8)
            assert abs(rep.iters - it8) <= 3, (rep.iters, it8)


def test_cg_3d():
    say("case cg 3d")
    probs = []
    for i, n in enumerate([12, 16]):
        g = np.random.default_rng(50 + i)
        m = g.uniform(2.0, 4.0, (n, n, n))
        c = np.exp(g.normal(0, 0.5, (n, n, n)))
        b = g.standard_normal((n, n, n))
        probs.append((n, m / n, c, b))
    rc, reps, xs = run(probs, ndl.NDL_F32C, dim=3, R=4, rtol=1e-8)
    assert rc == ndl.NDL_OK
    for (n, delta, c, b), rep, x in zip(probs, reps, xs):
        rr, _, _ = oracle_relres(n, delta, c, b, x, ndl.NDL_F32C, dim=3, R=4)
        assert rr <= 1.05e-8, rr


def test_cg_rejects_case_a():
    import torch
    n = 16
    d = torch.full((n, n), 3.0 / n, device="cuda")
    c = torch.ones((n, n), device="cuda")
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, 4, d, c, prec=ndl.NDL_F32C), keep=(d, c))
    b = torch.ones((n, n), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(ndl.NdlError) as e:
        ndl.ndl_cg_solve([plan], [b], [x])
    assert e.value.code == ndl.NDL_ENOTSPD


def test_cg_iteration_cap_reports_noconv():
    probs = problems([48])
    rc, reps, xs = run(probs, ndl.NDL_F64, rtol=1e-8, max_iter=5)
    assert rc == ndl.NDL_ENOCONV
    assert reps[0].converged == 0 and reps[0].iters <= 5 + 25


def test_learned_pcg_converges_and_falls_back():
    """Flexible PCG with the network (untrained here) still reaches 1e-8: the
    Jacobi fallback takes over on breakdown or stagnation."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    say("case learned pcg")
    n = 32
    plan, b, feat, w = PT.problem_3d(n, 3)
    net = ndl.ndl_net_create(seed=3)
    x = torch.zeros_like(b)
    rc, reps = ndl.ndl_cg_solve([plan], [b], [x], rtol=1e-8, precond=1, net=net)
    say("  rc", rc, "iters", reps[0].iters, "fell_back", reps[0].fell_back, "res", reps[0].rel_res_fp64)
    assert rc == ndl.NDL_OK and reps[0].converged
    P = O.Problem(dim=3, n=n, R=4, form="div", kernel="frac")
    d64 = w["delta"].astype(np.float32).astype(np.float64)
    c64 = w["coef"].astype(np.float32).astype(np.float64)
    xr = x.cpu().numpy()
    Ax = -O.apply(P, d64, c64, F.pad(xr, 4))
    bb = w["b"]
    assert np.linalg.norm(bb - Ax) / np.linalg.norm(bb) <= 1.05e-8


def test_precond_apply_is_finite_and_scale_covariant():
    import torch
    from paper_1905_08375_amd import precond_train as PT
    n = 32
    plan, b, feat, w = PT.problem_3d(n, 4)
    net = ndl.ndl_net_create(seed=4)
    r = torch.randn((n, n, n), device="cuda")
    z1 = torch.empty_like(r)
    z2 = torch.empty_like(r)
    ndl.ndl_precond_apply(net, plan, r, z1)
    ndl.ndl_precond_apply(net, plan, 4.0 * r, z2)
    torch.cuda.synchronize()
    assert torch.isfinite(z1).all()
    # z = ||r|| M(r / ||r||): scaling r scales z.  The factor is a power of two
    # so that r / ||r|| is bitwise the same for both calls (any other factor
    # perturbs it by an ulp, which can flip the BF16 rounding of an input).
    assert torch.allclose(z2, 4.0 * z1, rtol=1e-6, atol=1e-7 * float(z1.abs().max()))


def _shipped_net():
    from paper_1905_08375_amd import precond_train as PT
    import os
    if not os.path.exists(PT.WEIGHTS):
        pytest.skip("no trained weights in the tree")
    return PT.load_net(PT.WEIGHTS)


def test_linear_preconditioner_is_linear_and_starts_as_jacobi():
    """Linear mode: M(2r) = 2 M(r) exactly (powers of two pass through the
    BF16 network unchanged), M(r + s) ~ M(r) + M(s) to BF16 rounding, and a
    zeroed output layer gives M = 0, i.e. the two-level preconditioner is Jacobi."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    n = 32
    plan, b, feat, w = PT.problem_3d(n, 5)
    net = _shipped_net()
    g = torch.Generator(device="cuda").manual_seed(0)
    r = torch.randn((n, n, n), device="cuda", generator=g)
    t = torch.randn((n, n, n), device="cuda", generator=g)
    z1, z2, zt, zs = (torch.empty_like(r) for _ in range(4))
    ndl.ndl_precond_apply(net, plan, r, z1)
    ndl.ndl_precond_apply(net, plan, 2.0 * r, z2)
    ndl.ndl_precond_apply(net, plan, t, zt)
    ndl.ndl_precond_apply(net, plan, r + t, zs)
    torch.cuda.synchronize()
    assert torch.isfinite(z1).all() and float(z1.abs().max()) > 0
    assert torch.allclose(z2, 2.0 * z1, rtol=1e-6, atol=1e-7 * float(z1.abs().max()))
    lin_err = float((zs - z1 - zt).norm() / (z1 + zt).norm())
    say("  linearity defect", lin_err)
    assert lin_err < 0.05
    z0 = PT.new_net(seed=2)
    zz = torch.empty_like(r)
    ndl.ndl_precond_apply(z0, plan, r, zz)
    torch.cuda.synchronize()
    assert float(zz.abs().max()) == 0.0


@pytest.mark.parametrize("n", [64, 128, 256])
def test_trained_preconditioner_gains_over_jacobi(n):
    """The shipped network (trained on 256^3 fields of other seeds) in flexible
    PCG against plain Jacobi-CG on a held-out field: both reach a true FP64
    residual of 1e-8 (recomputed by the oracle over every node), the learned
    solve in far fewer iterations and without falling back.  n = 256 is the
    timed 3D solve itself (same field, seed and launch configuration)."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    say(f"case trained pcg n={n}")
    net = _shipped_net()
    plan, b, feat, w = PT.problem_3d(n, 100)
    x0 = torch.zeros_like(b)
    rc0, rep0 = ndl.ndl_cg_solve([plan], [b], [x0], rtol=1e-8)
    x1 = torch.zeros_like(b)
    rc1, rep1 = ndl.ndl_cg_solve([plan], [b], [x1], rtol=1e-8, precond=1, net=net)
    torch.cuda.synchronize()
    say("  plain", rep0[0].iters, "learned", rep1[0].iters, "fell_back", rep1[0].fell_back)
    assert rc0 == ndl.NDL_OK and rc1 == ndl.NDL_OK
    assert rep1[0].fell_back == 0
    assert rep1[0].iters <= 0.5 * rep0[0].iters
    P = O.Problem(dim=3, n=n, R=4, form="div", kernel="frac")
    d64 = w["delta"].astype(np.float32).astype(np.float64)
    c64 = w["coef"].astype(np.float32).astype(np.float64)
    for x in (x0, x1):
        xr = x.cpu().numpy()
        Ax = -O.apply(P, d64, c64, F.pad(xr, 4))
        assert np.linalg.norm(w["b"] - Ax) / np.linalg.norm(w["b"]) <= 1.05e-8


@pytest.mark.parametrize("lam", [-0.5, -4.0, -50.0])
def test_learned_pcg_recovers_from_an_indefinite_network(lam, tmp_path):
    """The shipped network with its output layer scaled by lam < 0 (so that
    r.z from the network can be negative): flexible PCG still reaches a true
    FP64 residual of 1e-8, recomputed by the oracle, through its Jacobi
    fallback (at the first direction or inside the loop, where the skipped
    step is retaken with the Jacobi z)."""
    import struct
    import torch
    from paper_1905_08375_amd import precond_train as PT
    say(f"case indefinite network lam={lam}")
    net = _shipped_net()
    path = tmp_path / "w.bin"
    ndl.ndl_net_save(net, str(path))
    raw = bytearray(path.read_bytes())
    pos, layers = 16, 13
    for i in range(layers):
        cout, kp = struct.unpack_from("<ii", raw, pos)
        pos += 8
        if i == layers - 1:
            w = np.frombuffer(bytes(raw[pos:pos + 4 * cout * kp]), dtype=np.float32) * np.float32(lam)
            raw[pos:pos + 4 * cout * kp] = w.astype(np.float32).tobytes()
        pos += 4 * cout * kp + 4 * cout
    assert pos == len(raw)
    path.write_bytes(bytes(raw))
    ndl.ndl_net_load(net, str(path))
    n = 32
    plan, b, feat, w = PT.problem_3d(n, 5)
    x = torch.zeros_like(b)
    rc, reps = ndl.ndl_cg_solve([plan], [b], [x], rtol=1e-8, precond=1, net=net)
    say("  rc", rc, "iters", reps[0].iters, "fell_back", reps[0].fell_back, "res", reps[0].rel_res_fp64)
    assert rc == ndl.NDL_OK and reps[0].converged
    if lam <= -50.0:
        assert reps[0].fell_back == 1
    P = O.Problem(dim=3, n=n, R=4, form="div", kernel="frac")
    d64 = w["delta"].astype(np.float32).astype(np.float64)
    c64 = w["coef"].astype(np.float32).astype(np.float64)
    Ax = -O.apply(P, d64, c64, F.pad(x.cpu().numpy(), 4))
    assert np.linalg.norm(w["b"] - Ax) / np.linalg.norm(w["b"]) <= 1.05e-8


def test_operator_cache_survives_plan_reuse():
    """The cached operator and Jacobi diagonal of the linear preconditioner
    belong to one plan: plans of other sizes created and destroyed in between
    (a new plan can take a destroyed plan's address) leave the result of a
    later plan unchanged, bit for bit."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    net = _shipped_net()
    n = 32
    g = torch.Generator(device="cuda").manual_seed(1)
    r = torch.randn((n, n, n), device="cuda", generator=g)

    def apply_fresh():
        plan, _, _, _ = PT.problem_3d(n, 3)
        z = torch.empty_like(r)
        ndl.ndl_precond_apply(net, plan, r, z)
        torch.cuda.synchronize()
        plan.close()
        return z

    ref = apply_fresh()
    for m in (16, 24, 8, 16):
        other, _, _, _ = PT.problem_3d(m, 4)
        zo = torch.empty((m, m, m), device="cuda")
        ndl.ndl_precond_apply(net, other, torch.randn((m, m, m), device="cuda", generator=g), zo)
        torch.cuda.synchronize()
        other.close()
        z = apply_fresh()
        assert torch.isfinite(z).all()
        assert torch.equal(z, ref), m


def test_batched_cg_on_the_full_workload():
    """The 64-instance workload itself, as the benchmark solves it (sizes drawn
    from 256^2..1024^2, 28.1M nodes, m in [2, 8], lognormal c, FP32
    compensated inner apply, FP64 refinement) in one call: the persistent item
    loop runs over far more tiles than the grid holds, problems of every size
    share the launch, and every instance's FP64 residual is recomputed over
    every node by the oracle."""
    import torch
    sizes = F.solve_sizes(64)
    say(f"case cg workload mix sizes={sizes}")
    assert len(set(sizes)) >= 4
    R = 8
    plans, bs, xs, ws = [], [], [], []
    for i, n in enumerate(sizes):
        w = F.solve_instance_2d(n, i)
        d_d, d_c = dev(w["delta"], ndl.NDL_F32C), dev(w["coef"], ndl.NDL_F32C)
        plans.append(ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, form=ndl.NDL_DIV, prec=ndl.NDL_F32C),
                                         keep=(d_d, d_c)))
        bs.append(torch.from_numpy(w["b"]).cuda())
        xs.append(torch.zeros((n, n), dtype=torch.float64, device="cuda"))
        ws.append(w)
    rc, reps = ndl.ndl_cg_solve(plans, bs, xs, rtol=1e-8)
    torch.cuda.synchronize()
    assert rc == ndl.NDL_OK, ndl.ndl_last_error()
    for i, (n, w, rep, x) in enumerate(zip(sizes, ws, reps, xs)):
        rr, _, _ = oracle_relres(n, w["delta"], w["coef"], w["b"], x.cpu().numpy(), ndl.NDL_F32C, R=R)
        say(f"  inst {i} n={n} iters={rep.iters} outer={rep.outer} gpu_res={rep.rel_res_fp64:.2e} oracle_res={rr:.2e}")
        assert rep.converged == 1
        assert rr <= 1.05e-8


def _div_batch(sizes, dim, prec, R, seed, mlo=2.0, mhi=8.0):
    import torch
    plans, xs, ws = [], [], []
    for i, n in enumerate(sizes):
        g = np.random.default_rng(seed + i)
        X = F.mesh(n, dim)
        ph = g.uniform(0, 1, size=2)
        m = (mlo + mhi) / 2 + (mhi - mlo) / 2 * np.sin(2 * np.pi * (X[0] + ph[0])) * np.cos(2 * np.pi * (X[-1] + ph[1]))
        c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
        x = g.standard_normal((n,) * dim)
        d_d, d_c = dev(m / n, prec), dev(c, prec)
        plans.append(ndl.ndl_plan_create(ndl.make_problem(dim, n, R, d_d, d_c, form=ndl.NDL_DIV, prec=prec),
                                         keep=(d_d, d_c)))
        xs.append(dev(x, prec))
        ws.append((m / n, c, x))
    return plans, xs, ws


@pytest.mark.parametrize("dim,prec,sizes,R,mhi", [
    (2, ndl.NDL_F32C, [768, 768, 512, 512, 512, 512, 300, 101, 37], 8, 8.0),
    (2, ndl.NDL_F64, [384, 200, 77], 8, 8.0),
    (3, ndl.NDL_F32C, [40, 33, 24], 4, 4.0),
])
def test_batched_apply_every_variant(dim, prec, sizes, R, mhi):
    """The solver's batched case (b) apply (one persistent launch over the tiles
    of uneven problems; in 2D more tiles than any grid holds) in every launch
    variant the autotuner may pick: each matches the FP64 oracle, all are
    bitwise alike, and the tuned choice is one of them."""
    import torch
    say(f"case batched apply variants dim={dim} prec={prec} sizes={sizes}")
    plans, xs, ws = _div_batch(sizes, dim, prec, R, 700 + dim, mhi=mhi)
    tdt = torch.float64 if prec == ndl.NDL_F64 else torch.float32
    refs = []
    for (delta, c, x), n in zip(ws, sizes):
        P = O.Problem(dim=dim, n=n, R=R, form="div", kernel="frac")
        npt = np.float64 if prec == ndl.NDL_F64 else np.float32
        refs.append(-O.apply(P, delta.astype(npt).astype(np.float64), c.astype(npt).astype(np.float64),
                             F.pad(x.astype(npt).astype(np.float64), R)))
    first, nvar = None, None
    v = 0
    while nvar is None or v < nvar:
        ys = [torch.full((n,) * dim, float("nan"), dtype=tdt, device="cuda") for n in sizes]
        used, nvar = ndl.ndl_div_batch_apply(plans, xs, ys, v)
        assert used == v
        got = [y.cpu().numpy() for y in ys]
        errs = [rel_l2(gg, rr) for gg, rr in zip(got, refs)]
        say(f"  variant {v}/{nvar} max rel l2 {max(errs):.2e}")
        assert max(errs) <= (1e-12 if prec == ndl.NDL_F64 else 1e-6)
        if first is None:
            first = got
        else:
            assert all(np.array_equal(a, b) for a, b in zip(got, first)), v
        v += 1
    assert nvar > 1
    ys = [torch.empty((n,) * dim, dtype=tdt, device="cuda") for n in sizes]
    used, _ = ndl.ndl_div_batch_apply(plans, xs, ys, -1)
    say(f"  tuned variant {used}")
    assert 0 <= used < nvar
    assert all(np.array_equal(y.cpu().numpy(), b) for y, b in zip(ys, first))


def test_batched_apply_3d_horizon_spikes():
    """The 3D batched case (b) apply ends each wave's offset loop at the largest
    horizon within reach of its block (its 32 columns and 4 rows widened by the
    reach, every plane within the reach).  A flat horizon m = 2 with isolated
    nodes of m = 3.9 (reach 3: m = 4 would round past k = 15 in FP32) at and
    beside those block edges, in the halo of a wave's block, on the grid's
    faces and in a ragged tile: every variant must still sum each spike's
    pairs (t = 8.7 against 4 for the flat field), element by element against
    the FP64 oracle."""
    import torch
    R = 4
    sizes = [70, 29]
    say(f"case 3D batched apply with horizon spikes sizes={sizes}")
    plans, xs, refs = [], [], []
    for i, n in enumerate(sizes):
        g = np.random.default_rng(880 + i)
        m = np.full((n, n, n), 2.0)
        cols = [c for c in (0, 1, 28, 29, 30, 31, 32, 33, 34, 35, 36, 63, 64, 66, 69) if c < n]
        for k, c in enumerate(cols):
            z, y = (5 * k + 3 * i) % n, (7 * k + 1) % n
            m[z, y, c] = 3.9
            m[(z + 9) % n, (y + 4) % n, c] = 3.9  # another plane and row block
        m[n - 1, n - 1, n - 1] = 3.9
        c = np.exp(g.normal(0.0, 0.5, (n,) * 3))
        x = g.standard_normal((n,) * 3)
        delta = (m / n).astype(np.float32)
        c32, x32 = c.astype(np.float32), x.astype(np.float32)
        d_d, d_c = dev(delta, ndl.NDL_F32C), dev(c32, ndl.NDL_F32C)
        plans.append(ndl.ndl_plan_create(ndl.make_problem(3, n, R, d_d, d_c, form=ndl.NDL_DIV, prec=ndl.NDL_F32C),
                                         keep=(d_d, d_c)))
        xs.append(dev(x32, ndl.NDL_F32C))
        P = O.Problem(dim=3, n=n, R=R, form="div", kernel="frac")
        refs.append(-O.apply(P, delta.astype(np.float64), c32.astype(np.float64),
                             F.pad(x32.astype(np.float64), R)))
    v, nvar = 0, None
    while nvar is None or v < nvar:
        ys = [torch.full((n,) * 3, float("nan"), dtype=torch.float32, device="cuda") for n in sizes]
        used, nvar = ndl.ndl_div_batch_apply(plans, xs, ys, v)
        assert used == v
        for y, ref, n in zip(ys, refs, sizes):
            got = y.cpu().numpy()
            err = rel_l2(got, ref)
            worst = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            say(f"  variant {v}/{nvar} n={n} rel l2 {err:.2e} worst node {worst:.2e}")
            assert err <= 1e-6 and worst <= 1e-5
        v += 1
