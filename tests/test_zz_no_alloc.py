"""ndl_apply_fast_noalloc (the hierarchical apply for callers that cannot
allocate: its pyramid lives in the library's static device workspace) against
ndl_apply_fast on the same inputs: two calls in a row, the second on a smaller
grid, and the size limit."""
import numpy as np
import pytest

from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import dev, say

pytestmark = pytest.mark.gpu


def _case(n, R, seed, prec):
    g = np.random.default_rng(seed)
    X = F.mesh(n, 2)
    m = 4.0 * (1.0 + 0.5 * np.sin(2 * np.pi * X[0] + seed) * np.cos(2 * np.pi * X[1]))
    c = np.exp(F.grf(n, 2, 0.5, 0.1, 9, seed))
    u = F.pad(F.grf(n, 2, 1.0, 0.1, 9, 100 + seed), R)
    return m / n, c, u


@pytest.mark.parametrize("prec", [ndl.NDL_F64, ndl.NDL_F32C])
def test_noalloc_fast_apply_equals_fast_apply(prec):
    import torch
    R = 6
    for n, seed, batch in [(1024, 1, 1), (203, 2, 2)]:
        say(f"case noalloc fast apply n={n} batch={batch} prec={prec}")
        delta, c, u = _case(n, R, seed, prec)
        d_d, d_c = dev(delta, prec), dev(c, prec)
        prob = ndl.make_problem(2, n, R, d_d, d_c, prec=prec)
        own = ndl.ndl_plan_create(prob, want_fast=1, keep=(d_d, d_c))
        bare = ndl.ndl_plan_create(prob, want_fast=2, keep=(d_d, d_c))
        du = dev(np.stack([u * (1 + b) for b in range(batch)]), prec)
        t = torch.float64 if prec == ndl.NDL_F64 else torch.float32
        ref = torch.zeros((batch, n, n), dtype=t, device="cuda")
        got = torch.full((batch, n, n), float("nan"), dtype=t, device="cuda")
        ndl.ndl_apply_fast(own, du, ref, batch)
        ndl.ndl_apply_fast_noalloc(bare, du, got, batch)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        # the plan without its own workspace runs only through the static one
        with pytest.raises(ndl.NdlError) as e:
            ndl.ndl_apply_fast(bare, du, ref, batch)
        assert e.value.code == ndl.NDL_EINVAL
        own.close()
        bare.close()


def test_noalloc_fast_apply_rejects_a_pyramid_beyond_the_workspace():
    import torch
    n, R = 8192, 2
    say(f"case noalloc size limit n={n}")
    d = torch.full((n, n), 1.5 / n, dtype=torch.float32, device="cuda")
    c = torch.ones((n, n), dtype=torch.float32, device="cuda")
    plan = ndl.ndl_plan_create(ndl.make_problem(2, n, R, d, c, kernel=ndl.NDL_G_CONST, prec=ndl.NDL_F32C),
                               want_fast=2, keep=(d, c))
    u = torch.zeros((n + 2 * R, n + 2 * R), dtype=torch.float32, device="cuda")
    out = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(ndl.NdlError) as e:
        ndl.ndl_apply_fast_noalloc(plan, u, out, 1)
    assert e.value.code == ndl.NDL_EINVAL
    assert "static workspace" in str(e.value)
    plan.close()
