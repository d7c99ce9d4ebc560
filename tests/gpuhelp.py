"""Helpers shared by the GPU parity tests (inputs, oracle calls, error norms)."""
import sys

import numpy as np

import oracle as O
from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl

KNAME = {ndl.NDL_G_CONST: "const", ndl.NDL_G_INV_R: "inv_r", ndl.NDL_G_FRAC: "frac", ndl.NDL_G_POLY: "poly",
         ndl.NDL_G_CONE: "cone"}
NNAME = {ndl.NDL_NORM_DISCRETE: "discrete", ndl.NDL_NORM_CONTINUOUS: "continuous", ndl.NDL_NORM_NONE: "none"}

TOL = {ndl.NDL_F64: 1e-12, ndl.NDL_F32C: 1e-6, ndl.NDL_F32K: 1e-6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return np.linalg.norm((got - ref).ravel()) / (den if den > 0 else 1.0)


def np_dtype(prec):
    return np.float64 if prec == ndl.NDL_F64 else np.float32


def torch_dtype(prec):
    import torch
    return torch.float64 if prec == ndl.NDL_F64 else torch.float32


def cast(a, prec):
    """Round to the path's storage type and return it as float64 (what the oracle reads)."""
    return np.asarray(a, dtype=np_dtype(prec)).astype(np.float64)


def dev(a, prec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np_dtype(prec)))).cuda()


def oracle_problem(dim, n, R, model, form, kernel, s, poly, norm):
    return O.Problem(dim=dim, n=n, R=R, model="peridynamic" if model == ndl.NDL_PERIDYNAMIC else "diffusion",
                     form={ndl.NDL_DIV: "div", ndl.NDL_SYM: "sym"}.get(form, "nd"), kernel=KNAME[kernel], s=s,
                     poly=list(poly), norm=NNAME[norm])


def gpu_apply(dim, n, R, delta, coef, u_pad, prec, *, model=ndl.NDL_DIFFUSION, form=ndl.NDL_ND,
              kernel=ndl.NDL_G_FRAC, s=0.5, poly=(1.0,), norm=ndl.NDL_NORM_DISCRETE, batch=None, fast=False):
    """Run ndl_apply (or ndl_apply_fast) through the C ABI; u_pad is [batch?][ncomp?][P..]."""
    import torch
    d_delta, d_coef = dev(delta, prec), dev(coef, prec)
    prob = ndl.make_problem(dim, n, R, d_delta, d_coef, model=model, form=form, kernel=kernel, s=s, poly=poly,
                            norm=norm, prec=prec)
    plan = ndl.ndl_plan_create(prob, want_fast=fast, keep=(d_delta, d_coef))
    ncomp = dim if model == ndl.NDL_PERIDYNAMIC else 1
    nb = 1 if batch is None else batch
    d_u = dev(u_pad, prec)
    out = torch.zeros((nb, ncomp) + (n,) * dim, dtype=torch_dtype(prec), device="cuda")
    (ndl.ndl_apply_fast if fast else ndl.ndl_apply)(plan, d_u, out, nb)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    info = plan.info()
    plan.close()
    if batch is None:
        res = res[0]
    if ncomp == 1:
        res = res[:, 0] if batch is not None else res[0]
    return res, info


def oracle_apply(dim, n, R, delta, coef, u_pad, prec, *, model=ndl.NDL_DIFFUSION, form=ndl.NDL_ND,
                 kernel=ndl.NDL_G_FRAC, s=0.5, poly=(1.0,), norm=ndl.NDL_NORM_DISCRETE):
    P = oracle_problem(dim, n, R, model, form, kernel, s, poly, norm)
    return O.apply(P, cast(delta, prec), cast(coef, prec), cast(u_pad, prec))


def rand_problem(dim, n, R, mlo, mhi, seed, smooth=False):
    g = np.random.default_rng(seed)
    if smooth:
        X = F.mesh(n, dim)
        m = mlo + (mhi - mlo) * 0.5 * (1 + np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[-1]))
    else:
        m = g.uniform(mlo, mhi, (n,) * dim)
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    u = F.pad(F.grf(n, dim, 1.0, 0.15, 77, seed) if n >= 4 else g.standard_normal((n,) * dim), R)
    # non-zero collar data (a volume constraint) for the direct paths
    if R > 0:
        mask = np.ones_like(u, dtype=bool)
        mask[tuple(slice(R, R + n) for _ in range(dim))] = False
        u[mask] = 0.3 * g.standard_normal(mask.sum())
    return m / n, c, u
