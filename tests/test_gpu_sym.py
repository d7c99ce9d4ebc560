"""The kernel-averaged symmetric form (ndl_apply, ndl_apply_fast, and CG
through ndl_cg_solve) against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import TOL, dev, gpu_apply, oracle_apply, rand_problem, rel_l2, say

pytestmark = pytest.mark.gpu

PRECS = [ndl.NDL_F64, ndl.NDL_F32C, ndl.NDL_F32K]
CASES = [
    (2, 90, 7, 2.0, 6.0, ndl.NDL_G_FRAC),
    (2, 61, 9, 3.0, 9.0, ndl.NDL_G_CONST),
    (1, 300, 20, 4.0, 20.0, ndl.NDL_G_INV_R),
    (3, 19, 4, 2.0, 4.0, ndl.NDL_G_FRAC),
    (3, 17, 5, 2.0, 5.0, ndl.NDL_G_CONST),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("dim,n,R,mlo,mhi,kernel", CASES)
def test_sym_apply(prec, fast, dim, n, R, mlo, mhi, kernel):
    """Direct sum and fast evaluation (case (a) hierarchical gather plus the
    adjoint scatter over row intervals) on ragged grids with collar data."""
    say(f"case sym dim={dim} n={n} kernel={kernel} fast={fast} prec={prec}")
    delta, c, u = rand_problem(dim, n, R, mlo, mhi, seed=1100 + n + dim, smooth=True)
    kw = dict(form=ndl.NDL_SYM, kernel=kernel)
    got, _ = gpu_apply(dim, n, R, delta, c, u, prec, fast=fast, **kw)
    ref = oracle_apply(dim, n, R, delta, c, u, prec, **kw)
    err = rel_l2(got, ref)
    say("  rel l2", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [ndl.NDL_F64, ndl.NDL_F32K])
def test_sym_apply_large_2d(prec):
    """The 2D direct sum on a grid large enough for its two-nodes-per-thread
    tiles (8 x 64; 730 leaves ragged rows and columns), with collar data,
    against the oracle."""
    dim, n, R = 2, 730, 7
    say(f"case sym large 2D n={n} prec={prec}")
    delta, c, u = rand_problem(dim, n, R, 2.0, 6.0, seed=1300, smooth=True)
    kw = dict(form=ndl.NDL_SYM, kernel=ndl.NDL_G_FRAC)
    got, _ = gpu_apply(dim, n, R, delta, c, u, prec, **kw)
    ref = oracle_apply(dim, n, R, delta, c, u, prec, **kw)
    err = rel_l2(got, ref)
    say("  rel l2", err)
    assert err <= TOL[prec]


def test_sym_cg_large_2d():
    """Jacobi-CG (FP64) through the two-nodes-per-thread direct sum and its
    diagonal at 730^2: the oracle's FP64 residual is <= 1e-8."""
    import torch
    dim, n, R = 2, 730, 7
    say(f"case sym cg large n={n}")
    g = np.random.default_rng(n)
    X = F.mesh(n, dim)
    m = 2.0 + 4.0 * 0.5 * (1 + np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[-1]))
    delta = m / n
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    b = g.standard_normal((n,) * dim)
    d_d, d_c = dev(delta, ndl.NDL_F64), dev(c, ndl.NDL_F64)
    plan = ndl.ndl_plan_create(ndl.make_problem(dim, n, R, d_d, d_c, form=ndl.NDL_SYM, kernel=ndl.NDL_G_FRAC,
                                                prec=ndl.NDL_F64), keep=(d_d, d_c))
    bb = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bb)
    rc, reps = ndl.ndl_cg_solve([plan], [bb], [x], rtol=1e-8)
    torch.cuda.synchronize()
    say(f"  rc {rc} iters {reps[0].iters} res {reps[0].rel_res_fp64:.2e}")
    assert rc == ndl.NDL_OK and reps[0].converged
    P = O.Problem(dim=dim, n=n, R=R, form="sym", kernel="frac")
    res = b + O.apply(P, delta, c, F.pad(x.cpu().numpy(), R))
    rel = np.linalg.norm(res) / np.linalg.norm(b)
    say(f"  oracle residual {rel:.2e}")
    assert rel <= 1.05e-8
    plan.close()


@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("dim,n,R,kernel", [(2, 24, 6, ndl.NDL_G_FRAC), (2, 28, 7, ndl.NDL_G_CONST),
                                            (3, 9, 4, ndl.NDL_G_FRAC)])
def test_sym_cg_against_a_dense_solve(fast, dim, n, R, kernel):
    """CG on -L_s (FP64, Jacobi) through the direct or the fast apply: the
    oracle's FP64 residual is <= 1e-8 and x agrees with a dense solve of the
    matrix assembled from the oracle within the residual-implied bound."""
    import torch
    say(f"case sym cg dim={dim} n={n} kernel={kernel} fast={fast}")
    g = np.random.default_rng(n + dim)
    X = F.mesh(n, dim)
    m = 2.0 + (R - 2.0) * 0.5 * (1 + np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[-1]))
    delta = m / n
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    b = g.standard_normal((n,) * dim)
    d_d, d_c = dev(delta, ndl.NDL_F64), dev(c, ndl.NDL_F64)
    plan = ndl.ndl_plan_create(ndl.make_problem(dim, n, R, d_d, d_c, form=ndl.NDL_SYM, kernel=kernel,
                                                prec=ndl.NDL_F64), want_fast=int(fast), keep=(d_d, d_c))
    bb = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bb)
    rc, reps = ndl.ndl_cg_solve([plan], [bb], [x], rtol=1e-8, use_fast=fast)
    torch.cuda.synchronize()
    say(f"  rc {rc} iters {reps[0].iters} res {reps[0].rel_res_fp64:.2e}")
    assert rc == ndl.NDL_OK and reps[0].converged
    P = O.Problem(dim=dim, n=n, R=R, form="sym", kernel={ndl.NDL_G_FRAC: "frac", ndl.NDL_G_CONST: "const"}[kernel])
    xs = x.cpu().numpy()
    res = b + O.apply(P, delta, c, F.pad(xs, R))
    rel = np.linalg.norm(res) / np.linalg.norm(b)
    say(f"  oracle residual {rel:.2e}")
    assert rel <= 1.05e-8
    N = n ** dim
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros((n,) * dim)
        e.flat[j] = 1.0
        A[:, j] = -O.apply(P, delta, c, F.pad(e, R)).ravel()
    xd = np.linalg.solve(A, b.ravel())
    cond = np.linalg.cond(A)
    assert np.linalg.norm(xs.ravel() - xd) <= 2 * cond * 1.05e-8 * np.linalg.norm(xd)
    plan.close()


def test_sym_rejects_unsupported():
    import torch
    n = 16
    d = torch.full((n, n), 3.0 / n, dtype=torch.float64, device="cuda")
    c = torch.ones((n, n), dtype=torch.float64, device="cuda")
    for kw in [dict(kernel=ndl.NDL_G_POLY), dict(kernel=ndl.NDL_G_CONE), dict(model=ndl.NDL_PERIDYNAMIC)]:
        with pytest.raises(ndl.NdlError) as e:
            ndl.ndl_plan_create(ndl.make_problem(2, n, 4, d, c, form=ndl.NDL_SYM, prec=ndl.NDL_F64, **kw), keep=(d, c))
        assert e.value.code == ndl.NDL_EUNSUPPORTED
