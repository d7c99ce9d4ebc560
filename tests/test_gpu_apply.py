"""GPU parity of ndl_apply / ndl_apply_fast (through the C ABI) against the FP64 oracle.

Bars: relative L2 error <= 1e-12 for FP64, <= 1e-6 for FP32 storage with
FP64-carried (F32C) or Kahan-compensated FP32 (F32K) sums; the oracle reads the
same FP32-rounded inputs promoted to FP64."""
import numpy as np
import pytest

import oracle as O
from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import TOL, gpu_apply, oracle_apply, rand_problem, rel_l2, say, cast

pytestmark = pytest.mark.gpu
PRECS = [ndl.NDL_F64, ndl.NDL_F32C, ndl.NDL_F32K]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [100, 37])
def test_2d_nd_frac_random_horizon(prec, n):
    say(f"case 2d nd frac n={n} prec={prec}")
    R = 6
    delta, c, u = rand_problem(2, n, R, 2.0, 6.0, seed=n)
    got, info = gpu_apply(2, n, R, delta, c, u, prec)
    ref = oracle_apply(2, n, R, delta, c, u, prec)
    err = rel_l2(got, ref)
    say("  rel l2", err, "kmax", info.k_max)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel,norm,s,poly", [
    (ndl.NDL_G_CONST, ndl.NDL_NORM_DISCRETE, 0.5, (1.0,)),
    (ndl.NDL_G_INV_R, ndl.NDL_NORM_DISCRETE, 0.5, (1.0,)),
    (ndl.NDL_G_FRAC, ndl.NDL_NORM_CONTINUOUS, 0.25, (1.0,)),
    (ndl.NDL_G_CONST, ndl.NDL_NORM_NONE, 0.5, (1.0,)),
    (ndl.NDL_G_POLY, ndl.NDL_NORM_DISCRETE, 0.5, (2.1875, -2.1875, 1.3125, -0.3125)),
    (ndl.NDL_G_POLY, ndl.NDL_NORM_CONTINUOUS, 0.5, (1.5, -0.5)),
])
def test_2d_nd_profiles(prec, kernel, norm, s, poly):
    say(f"case 2d profile k={kernel} norm={norm} prec={prec}")
    n, R = 45, 5
    delta, c, u = rand_problem(2, n, R, 1.5, 5.5, seed=7)
    kw = dict(kernel=kernel, norm=norm, s=s, poly=poly)
    got, _ = gpu_apply(2, n, R, delta, c, u, prec, **kw)
    ref = oracle_apply(2, n, R, delta, c, u, prec, **kw)
    assert rel_l2(got, ref) <= TOL[prec]


def test_1d_config_sines():
    """1D, n = 4096, delta = 0.01, constant kernel 3/delta^3 (continuous normalisation), FP64."""
    say("case 1d sines")
    d = F.diffusion_1d()
    n, R = 4096, 41
    u = F.pad(d["u"], R)
    kw = dict(kernel=ndl.NDL_G_CONST, norm=ndl.NDL_NORM_CONTINUOUS)
    got, info = gpu_apply(1, n, R, d["delta"], d["coef"], u, ndl.NDL_F64, **kw)
    ref = oracle_apply(1, n, R, d["delta"], d["coef"], u, ndl.NDL_F64, **kw)
    assert info.k_max == 1677
    assert rel_l2(got, ref) <= 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_1d_random(prec):
    n, R = 333, 12
    delta, c, u = rand_problem(1, n, R, 1.0, 12.0, seed=3)
    got, _ = gpu_apply(1, n, R, delta, c, u, prec)
    ref = oracle_apply(1, n, R, delta, c, u, prec)
    assert rel_l2(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_1d_batched_ragged(prec):
    """1D nodes share their pair loop among lanes; a ragged last tile and a batch."""
    say(f"case 1d batched prec={prec}")
    n, R, B = 77, 20, 3
    delta, c, _ = rand_problem(1, n, R, 2.0, 20.0, seed=13)
    g = np.random.default_rng(14)
    u = g.standard_normal((B, n + 2 * R))
    got, _ = gpu_apply(1, n, R, delta, c, u, prec, batch=B)
    for b in range(B):
        ref = oracle_apply(1, n, R, delta, c, u[b], prec)
        assert rel_l2(got[b], ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_3d_nd(prec):
    say(f"case 3d nd prec={prec}")
    n, R = 21, 4
    delta, c, u = rand_problem(3, n, R, 2.0, 4.0, seed=5)
    got, _ = gpu_apply(3, n, R, delta, c, u, prec)
    ref = oracle_apply(3, n, R, delta, c, u, prec)
    assert rel_l2(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_pd_batched(prec):
    say(f"case pd prec={prec}")
    n, R, B = 70, 12, 3
    g = np.random.default_rng(11)
    delta = g.uniform(3.0, 12.0, (n, n)) / n
    c = g.uniform(0.5, 2.0, (n, n))
    u = np.stack([np.stack([F.pad(F.grf(n, 2, 1e-3, 0.1, 9, 2 * b + q), R) for q in range(2)]) for b in range(B)])
    u += 1e-3 * g.standard_normal(u.shape)  # collar data too
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_INV_R)
    got, _ = gpu_apply(2, n, R, delta, c, u, prec, batch=B, **kw)
    for b in range(B):
        ref = oracle_apply(2, n, R, delta, c, u[b], prec, **kw)
        err = rel_l2(got[b], ref)
        say("  field", b, "rel l2", err)
        assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", [ndl.NDL_G_FRAC, ndl.NDL_G_CONST])
def test_2d_wide_horizon_every_variant(prec, kernel):
    """2D diffusion with horizons of 8 to 21 nodes (past the unrolled tables:
    the run-time-horizon kernel) on a ragged grid: every tile matches the
    oracle and all are bitwise alike."""
    import torch
    from gpuhelp import dev
    say(f"case 2d wide prec={prec} kernel={kernel}")
    n, R = 100, 22
    delta, c, u = rand_problem(2, n, R, 8.0, 21.0, seed=55)
    kw = dict(kernel=kernel)
    ref = oracle_apply(2, n, R, delta, c, u, prec, **kw)
    d_d, d_c, d_u = dev(delta, prec), dev(c, prec), dev(u, prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, kernel=kernel, prec=prec), keep=(d_d, d_c))
    out = torch.zeros((n, n), dtype=d_u.dtype, device="cuda")
    first = None
    for v in range(ndl.ndl_plan_num_variants(plan)):
        ndl.ndl_plan_set_variant(plan, v)
        assert plan.info().pair_order == 2
        out.zero_()
        ndl.ndl_apply(plan, d_u, out, 1)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        err = rel_l2(o, ref)
        assert err <= TOL[prec], (v, err)
        first = o if first is None else first
        assert np.array_equal(o, first), v


@pytest.mark.parametrize("prec", PRECS)
def test_pd_every_tile_variant(prec):
    """Peridynamics on a ragged 2D grid (horizon up to 12 nodes): every tile the
    autotuner may pick matches the oracle, all bitwise alike (one pair order)."""
    import torch
    from gpuhelp import dev
    say(f"case pd variants prec={prec}")
    n, R, B = 83, 12, 2
    g = np.random.default_rng(12)
    X = F.mesh(n, 2)
    delta = (7.5 + 4.5 * np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1])) / n
    c = g.uniform(0.5, 2.0, (n, n))
    u = np.stack([np.stack([F.pad(F.grf(n, 2, 1e-3, 0.1, 9, 5 * b + q), R) for q in range(2)]) for b in range(B)])
    u += 1e-4 * g.standard_normal(u.shape)
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_INV_R)
    refs = [oracle_apply(2, n, R, delta, c, u[b], prec, **kw) for b in range(B)]
    d_d, d_c, d_u = dev(delta, prec), dev(c, prec), dev(u, prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, model=ndl.NDL_PERIDYNAMIC,
                                                kernel=ndl.NDL_G_INV_R, prec=prec), keep=(d_d, d_c))
    out = torch.zeros((B, 2, n, n), dtype=d_u.dtype, device="cuda")
    first = None
    for v in range(ndl.ndl_plan_num_variants(plan)):
        ndl.ndl_plan_set_variant(plan, v)
        out.zero_()
        ndl.ndl_apply(plan, d_u, out, B)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        for b in range(B):
            assert rel_l2(o[b], refs[b]) <= TOL[prec], (v, b)
        first = o if first is None else first
        assert np.array_equal(o, first), v
        assert plan.info().pair_order == 1


def test_pd_full_workload():
    """The peridynamic workload at its full size, as the benchmark runs it
    (2048^2, 8 displacement fields in one launch, m in [3, 12], Voronoi c,
    FP32 with Kahan sums, the tile tuned on these fields at batch 8): the
    first and last fields against the oracle."""
    import torch
    from gpuhelp import dev
    prec = ndl.NDL_F32K
    w = F.peridynamic_2d()
    n, R, B = 2048, 12, 8
    say(f"case pd full workload n={n} batch={B}")
    d_d, d_c, d_u = dev(w["delta"], prec), dev(w["coef"], prec), dev(w["u"], prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, model=ndl.NDL_PERIDYNAMIC,
                                                kernel=ndl.NDL_G_INV_R, prec=prec), keep=(d_d, d_c))
    ndl.ndl_autotune_apply(plan, d_u, B)
    out = torch.zeros((B, 2, n, n), dtype=d_u.dtype, device="cuda")
    ndl.ndl_apply(plan, d_u, out, B)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_INV_R)
    for b in (0, B - 1):
        ref = oracle_apply(2, n, R, w["delta"], w["coef"], w["u"][b], prec, **kw)
        err = rel_l2(o[b], ref)
        say(f"  field {b} variant {plan.info().variant} rel l2 {err:.3e}")
        assert err <= TOL[prec], b
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,n,R", [(2, 70, 8), (3, 18, 4), (1, 200, 9)])
def test_div(prec, dim, n, R):
    say(f"case div dim={dim} prec={prec}")
    mhi = {1: 9.0, 2: 8.0, 3: 4.0}[dim]
    delta, c, u = rand_problem(dim, n, R, 2.0, mhi, seed=13 + dim)
    kw = dict(form=ndl.NDL_DIV)
    got, _ = gpu_apply(dim, n, R, delta, c, u, prec, **kw)
    ref = oracle_apply(dim, n, R, delta, c, u, prec, **kw)
    assert rel_l2(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_div_1d_batched_ragged(prec):
    """1D case (b): nodes share their pair loop among lanes; ragged tile, batch."""
    say(f"case div 1d batched prec={prec}")
    n, R, B = 333, 12, 2
    delta, c, _ = rand_problem(1, n, R, 2.0, 12.0, seed=21)
    g = np.random.default_rng(22)
    u = g.standard_normal((B, n + 2 * R))
    got, _ = gpu_apply(1, n, R, delta, c, u, prec, form=ndl.NDL_DIV, batch=B)
    for b in range(B):
        ref = oracle_apply(1, n, R, delta, c, u[b], prec, form=ndl.NDL_DIV)
        assert rel_l2(got[b], ref) <= TOL[prec]


def test_div_continuous_and_const():
    n, R = 40, 6
    delta, c, u = rand_problem(2, n, R, 2.0, 6.0, seed=17)
    for kernel, norm in [(ndl.NDL_G_FRAC, ndl.NDL_NORM_CONTINUOUS), (ndl.NDL_G_CONST, ndl.NDL_NORM_NONE)]:
        kw = dict(form=ndl.NDL_DIV, kernel=kernel, norm=norm)
        got, _ = gpu_apply(2, n, R, delta, c, u, ndl.NDL_F64, **kw)
        ref = oracle_apply(2, n, R, delta, c, u, ndl.NDL_F64, **kw)
        assert rel_l2(got, ref) <= 1e-12


# ------------------------------------------------------------------ edge cases
def test_single_node_and_zero_horizon():
    for n, m in [(1, 0.5), (1, 3.0), (5, 0.9)]:
        R = 3
        delta = np.full((n, n), m / n)
        c = np.ones((n, n))
        u = np.random.default_rng(1).standard_normal((n + 2 * R,) * 2)
        got, info = gpu_apply(2, n, R, delta, c, u, ndl.NDL_F64, kernel=ndl.NDL_G_CONST, norm=ndl.NDL_NORM_NONE)
        ref = oracle_apply(2, n, R, delta, c, u, ndl.NDL_F64, kernel=ndl.NDL_G_CONST, norm=ndl.NDL_NORM_NONE)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("form", [ndl.NDL_ND, ndl.NDL_DIV])
def test_1d_grids_smaller_than_a_tile(form):
    """1D grids of 1, 3 and 17 nodes (below one 16-node tile, and one past it),
    partners reaching into the collar on both sides."""
    for n, m in [(1, 0.5), (1, 2.5), (3, 2.0), (17, 4.0)]:
        R = 4
        delta, c, _ = rand_problem(1, n, R, 0.5 * m, m, seed=30 + n)
        u = np.random.default_rng(31 + n).standard_normal(n + 2 * R)
        kw = dict(form=form, kernel=ndl.NDL_G_CONST, norm=ndl.NDL_NORM_NONE)
        got, _ = gpu_apply(1, n, R, delta, c, u, ndl.NDL_F64, **kw)
        ref = oracle_apply(1, n, R, delta, c, u, ndl.NDL_F64, **kw)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-300), (n, m)


def test_collar_too_small_is_an_error():
    import torch
    n = 16
    d = torch.full((n, n), 5.5 / n, dtype=torch.float64, device="cuda")  # k = 30 needs R >= 5
    c = torch.ones((n, n), dtype=torch.float64, device="cuda")
    prob = ndl.make_problem(2, n, 4, d, c, prec=ndl.NDL_F64)
    with pytest.raises(ndl.NdlError) as e:
        ndl.ndl_plan_create(prob)
    assert e.value.code == ndl.NDL_EINVAL


def test_batch_zero_is_a_no_op():
    import torch
    n, R = 8, 3
    d = torch.full((n, n), 2.5 / n, dtype=torch.float32, device="cuda")
    c = torch.ones((n, n), dtype=torch.float32, device="cuda")
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, prec=ndl.NDL_F32C), keep=(d, c))
    u = torch.zeros((1, n + 2 * R, n + 2 * R), device="cuda")
    out = torch.full((1, n, n), 7.0, device="cuda")
    ndl.ndl_apply(plan, u, out, 0)
    torch.cuda.synchronize()
    assert float(out[0, 0, 0]) == 7.0


# ------------------------------------------------------------------ config sizes
@pytest.mark.parametrize("prec", PRECS)
def test_config_2d_1024_full(prec):
    """The 2D workload: 1024^2, m(x) = 4(1 + 0.5 sin 2 pi x1 cos 2 pi x2), lognormal c, GRF u."""
    import torch
    from gpuhelp import dev
    say(f"case c2 full prec={prec}")
    w = F.diffusion_2d()
    n, R = 1024, 6
    u = F.pad(w["u"], R)
    ref = oracle_apply(2, n, R, w["delta"], w["coef"], u, prec)
    d_d, d_c, d_u = dev(w["delta"], prec), dev(w["coef"], prec), dev(u, prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, prec=prec), keep=(d_d, d_c))
    out = torch.zeros((n, n), dtype=d_u.dtype, device="cuda")
    # the tile the autotuner picks (the benchmarked launch), then every other tile
    ndl.ndl_autotune(plan)
    chosen = plan.info().variant
    for v in [chosen] + [v for v in range(ndl.ndl_plan_num_variants(plan)) if v != chosen]:
        ndl.ndl_plan_set_variant(plan, v)
        out.zero_()
        ndl.ndl_apply(plan, d_u, out, 1)
        torch.cuda.synchronize()
        info = plan.info()
        err = rel_l2(out.cpu().numpy(), ref)
        say("  variant", v, "tile", info.tile_x, info.tile_y, "rel l2", err, "kmax", info.k_max, "kmin", info.k_min)
        assert err <= TOL[prec], v


# ------------------------------------------------------------------ Section 3 path
def zero_collar(u, R, dim):
    v = np.zeros_like(u)
    sl = tuple(slice(R, u.shape[a] - R) for a in range(dim))
    v[sl] = u[sl]
    return v


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,n,R,mlo,mhi,kernel,norm", [
    (2, 100, 6, 2.0, 6.0, ndl.NDL_G_FRAC, ndl.NDL_NORM_DISCRETE),
    (2, 64, 33, 31.0, 33.0, ndl.NDL_G_CONST, ndl.NDL_NORM_NONE),
    (2, 50, 12, 4.0, 12.0, ndl.NDL_G_INV_R, ndl.NDL_NORM_DISCRETE),
    (1, 300, 40, 5.0, 40.0, ndl.NDL_G_CONST, ndl.NDL_NORM_CONTINUOUS),
    (3, 20, 5, 2.0, 5.0, ndl.NDL_G_FRAC, ndl.NDL_NORM_DISCRETE),
])
def test_fast_equals_direct_oracle(prec, dim, n, R, mlo, mhi, kernel, norm):
    say(f"case fast dim={dim} n={n} k={kernel} prec={prec}")
    delta, c, u = rand_problem(dim, n, R, mlo, mhi, seed=29 + n, smooth=True)
    u = zero_collar(u, R, dim)
    kw = dict(kernel=kernel, norm=norm)
    got, info = gpu_apply(dim, n, R, delta, c, u, prec, fast=True, **kw)
    ref = oracle_apply(dim, n, R, delta, c, u, prec, **kw)
    err = rel_l2(got, ref)
    say("  rel l2", err, "levels", info.fast_levels)
    assert err <= TOL[prec]


def test_fast_example1_regime():
    """Example 1: delta = 1/2, C = 1, p^0 = 1, zero volume constraint; here n = 128."""
    say("case example1")
    n = 128
    R = n // 2 + 1
    delta = np.full((n, n), 0.5)
    c = np.ones((n, n))
    g = np.random.default_rng(3)
    u = zero_collar(F.pad(g.standard_normal((n, n)), R), R, 2)
    kw = dict(kernel=ndl.NDL_G_CONST, norm=ndl.NDL_NORM_NONE)
    got, info = gpu_apply(2, n, R, delta, c, u, ndl.NDL_F64, fast=True, **kw)
    P = O.Problem(dim=2, n=n, R=R, kernel="const", norm="none")
    ref = O.fast_apply_const(P, delta, c, u[R:-R, R:-R])
    assert rel_l2(got, ref) <= 1e-12


def test_device_decomposition_matches_oracle():
    import torch
    n = 48
    g = np.random.default_rng(4)
    m = g.uniform(2.0, 20.0, (n, n))
    d = torch.from_numpy(m / n).cuda()
    c = torch.ones((n, n), dtype=torch.float64, device="cuda")
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, 21, d, c, prec=ndl.NDL_F64, kernel=ndl.NDL_G_CONST),
                               want_fast=True, keep=(d, c))
    # the tree covers the padded box: the node sits at node + R in a domain of n + 2R
    R = 21
    P = n + 2 * R
    L = O.tree_levels(P)
    for node in [(0, 0), (47, 47), (10, 30), (24, 24), (3, 44)]:
        k = O.cutoff(m[node] / n, n)
        got = sorted((L - s, j) for s, j in ndl.ndl_fast_decomposition(plan, node))
        assert got == sorted(O.decompose(2, P, (node[0] + R, node[1] + R), k))


@pytest.mark.parametrize("prec", PRECS)
def test_every_tile_variant_and_autotune(prec):
    """Each tile variant the autotuner may pick matches the oracle, and variants
    with the same pair order give bitwise the same result (the per-node
    summation order depends on the order, not on the tile)."""
    import torch
    say(f"case variants prec={prec}")
    n, R = 150, 6
    delta, c, u = rand_problem(2, n, R, 2.0, 6.0, seed=41, smooth=True)
    from gpuhelp import dev, torch_dtype
    d_d, d_c, d_u = dev(delta, prec), dev(c, prec), dev(u, prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, prec=prec), keep=(d_d, d_c))
    nv = ndl.ndl_plan_num_variants(plan)
    assert nv >= 2
    outs, orders = [], []
    for v in range(nv):
        ndl.ndl_plan_set_variant(plan, v)
        orders.append(plan.info().pair_order)
        o = torch.zeros((n, n), dtype=torch_dtype(prec), device="cuda")
        ndl.ndl_apply(plan, d_u, o, 1)
        outs.append(o.cpu().numpy())
    assert set(orders) == {0, 1}
    ref = oracle_apply(2, n, R, delta, c, u, prec)
    first = {}
    for v, o in enumerate(outs):
        assert rel_l2(o, ref) <= TOL[prec], v
        first.setdefault(orders[v], o)
        assert np.array_equal(o, first[orders[v]]), v
    info = ndl.ndl_autotune(plan)
    assert 0 <= info.variant < nv
    with pytest.raises(ndl.NdlError):
        ndl.ndl_plan_set_variant(plan, nv)


@pytest.mark.parametrize("fast", [False, True])
def test_graph_replay_matches_eager(fast):
    """The applies contain no allocation, copy or fill, so they can be captured
    in a HIP graph (as the benchmark times them): every replay, with eager work
    and synchronisations in between, gives bitwise the eager result."""
    import torch
    from gpuhelp import dev
    say(f"case graph replay fast={fast}")
    n, R = 130, 6
    prec = ndl.NDL_F32K if not fast else ndl.NDL_F32C
    delta, c, u = rand_problem(2, n, R, 2.0, 6.0, seed=77, smooth=True)
    d_d, d_c, d_u = dev(delta, prec), dev(c, prec), dev(u, prec)
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, prec=prec), want_fast=int(fast), keep=(d_d, d_c))
    out = torch.zeros((n, n), dtype=d_u.dtype, device="cuda")
    fn = (lambda: ndl.ndl_apply_fast(plan, d_u, out, 1)) if fast else (lambda: ndl.ndl_apply(plan, d_u, out, 1))
    fn()
    torch.cuda.synchronize()
    eager = out.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
        fn()
    for rep in range(4):
        out.zero_()
        scratch = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert torch.isfinite(scratch)
    ref = oracle_apply(2, n, R, delta, c, u, prec)
    assert rel_l2(out.cpu().numpy(), ref) <= TOL[prec]


@pytest.mark.parametrize("m", [4.0, 70.0])
def test_pairs_per_point_is_the_average_ball(m):
    """The plan's pairs_per_point is the mean over nodes of the lattice-ball
    size #{z != 0 : |z|^2 <= k_i}, k_i = ceil((delta_i n)^2) - 1 from the FP32
    horizon in FP64; m = 4 bins the cutoffs in LDS, m = 70 (k up to 7655)
    in the global bins."""
    import torch
    say(f"case pairs_per_point m={m}")
    n = 256
    X = F.mesh(n, 2)
    mm = m * (1.0 + 0.25 * np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1]))
    delta = (mm / n).astype(np.float32)
    R = int(np.ceil(mm.max())) + 1
    d_d = torch.from_numpy(delta).cuda()
    d_c = torch.ones((n, n), dtype=torch.float32, device="cuda")
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d_d, d_c, prec=ndl.NDL_F32K), keep=(d_d, d_c))
    got = plan.info().pairs_per_point
    plan.close()
    k = (np.ceil((delta.astype(np.float64) * n) ** 2) - 1).astype(np.int64)
    kmax = int(k.max())
    J = int(np.sqrt(kmax)) + 1
    a = np.arange(-J, J + 1)
    q = (a[:, None] ** 2 + a[None, :] ** 2).ravel()
    q = q[(q > 0) & (q <= kmax)]
    ball = np.cumsum(np.bincount(q, minlength=kmax + 1))
    want = ball[k].mean()
    say("  pairs_per_point", got, "expected", want, "kmax", kmax)
    assert abs(got - want) <= 1e-12 * want
