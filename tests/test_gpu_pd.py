"""Peridynamics in 3D (three displacement components) and the conical
micromodulus (1 - r)/r of eq. "kernelgamma" through the C ABI, against the
FP64 oracle."""
import numpy as np
import pytest

from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import TOL, gpu_apply, oracle_apply, rand_problem, rel_l2, say

pytestmark = pytest.mark.gpu

PRECS = [ndl.NDL_F64, ndl.NDL_F32C, ndl.NDL_F32K]


def _pd3_fields(n, R, B, mlo, mhi, seed):
    g = np.random.default_rng(seed)
    X = F.mesh(n, 3)
    m = mlo + (mhi - mlo) * 0.5 * (1 + np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1]) * np.sin(np.pi * X[2]))
    c = g.uniform(0.5, 2.0, (n, n, n))
    Xp = F.padded_coords(n, 3, R)
    us = []
    for b in range(B):
        W = 1e-3 * g.standard_normal((3, 3))
        W = W - W.T  # infinitesimal rotation
        rot = np.stack([sum(W[a, q] * (Xp[q] - 0.5) for q in range(3)) for a in range(3)])
        rnd = np.stack([F.pad(F.grf(n, 3, 1e-3, 0.15, 9, 11 * b + q), R) for q in range(3)])
        us.append(rot + rnd + 1e-4 * g.standard_normal(rot.shape))  # collar data too
    return m / n, c, np.stack(us)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kernel", [ndl.NDL_G_INV_R, ndl.NDL_G_FRAC, ndl.NDL_G_CONE])
def test_pd_3d_direct(prec, kernel):
    """3D peridynamics, horizons of 2 to 4 nodes on a ragged 23^3 grid, a
    batch of 2 fields (rotation plus a random field, collar data)."""
    say(f"case pd3 direct kernel={kernel} prec={prec}")
    n, R, B = 23, 4, 2
    delta, c, u = _pd3_fields(n, R, B, 2.0, 4.0, 70 + kernel)
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=kernel)
    got, _ = gpu_apply(3, n, R, delta, c, u, prec, batch=B, **kw)
    for b in range(B):
        ref = oracle_apply(3, n, R, delta, c, u[b], prec, **kw)
        err = rel_l2(got[b], ref)
        say("  field", b, "rel l2", err)
        assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_pd_3d_fast(prec):
    """3D peridynamics through the hierarchical path (degree-2 moments of the
    three components, the remainder summed directly)."""
    say(f"case pd3 fast prec={prec}")
    n, R, B = 22, 5, 1
    delta, c, u = _pd3_fields(n, R, B, 2.0, 5.0, 81)
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_INV_R)
    got, info = gpu_apply(3, n, R, delta, c, u, prec, batch=B, fast=True, **kw)
    ref = oracle_apply(3, n, R, delta, c, u[0], prec, **kw)
    err = rel_l2(got[0], ref)
    say("  rel l2", err, "levels", info.fast_levels)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim,n,R,mlo,mhi,norm", [
    (1, 200, 12, 3.0, 12.0, ndl.NDL_NORM_DISCRETE),
    (2, 70, 9, 2.0, 9.0, ndl.NDL_NORM_CONTINUOUS),
    (2, 64, 6, 2.0, 6.0, ndl.NDL_NORM_NONE),
    (3, 17, 4, 2.0, 4.0, ndl.NDL_NORM_DISCRETE),
])
def test_cone_diffusion_direct(prec, dim, n, R, mlo, mhi, norm):
    """The conical profile for nonlocal diffusion (case (a)), every normalisation."""
    say(f"case cone diffusion dim={dim} prec={prec}")
    delta, c, u = rand_problem(dim, n, R, mlo, mhi, seed=90 + dim, smooth=True)
    kw = dict(kernel=ndl.NDL_G_CONE, norm=norm)
    got, _ = gpu_apply(dim, n, R, delta, c, u, prec, **kw)
    ref = oracle_apply(dim, n, R, delta, c, u, prec, **kw)
    err = rel_l2(got, ref)
    say("  rel l2", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_cone_pd_2d_direct(prec):
    """2D peridynamics with the conical micromodulus (the generic kernel)."""
    say(f"case cone pd2 prec={prec}")
    n, R = 61, 10
    g = np.random.default_rng(5)
    X = F.mesh(n, 2)
    delta = (6.0 + 4.0 * np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1])) / n
    c = g.uniform(0.5, 2.0, (n, n))
    u = np.stack([F.pad(F.grf(n, 2, 1e-3, 0.1, 9, 40 + q), R) for q in range(2)])
    u += 1e-4 * g.standard_normal(u.shape)
    kw = dict(model=ndl.NDL_PERIDYNAMIC, kernel=ndl.NDL_G_CONE)
    got, _ = gpu_apply(2, n, R, delta, c, u, prec, **kw)
    ref = oracle_apply(2, n, R, delta, c, u, prec, **kw)
    err = rel_l2(got, ref)
    say("  rel l2", err)
    assert err <= TOL[prec]


def test_cone_rejected_where_unsupported():
    import torch
    n = 16
    d = torch.full((n, n), 3.0 / n, dtype=torch.float64, device="cuda")
    c = torch.ones((n, n), dtype=torch.float64, device="cuda")
    for kw, fast in [(dict(form=ndl.NDL_DIV), 0), (dict(), 1)]:
        with pytest.raises(ndl.NdlError) as e:
            ndl.ndl_plan_create(ndl.make_problem(2, n, 4, d, c, kernel=ndl.NDL_G_CONE, prec=ndl.NDL_F64, **kw),
                                want_fast=fast, keep=(d, c))
        assert e.value.code == ndl.NDL_EUNSUPPORTED
