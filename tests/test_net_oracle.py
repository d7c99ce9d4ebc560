"""Pins of the network oracle (CPU): adjoint identity, finite differences,
an independent library correlation, and BF16 rounding against torch."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import net_oracle as NO


def test_bf16_rounding_matches_torch():
    import torch
    g = np.random.default_rng(0)
    a = np.concatenate([g.standard_normal(1000) * 10.0 ** g.integers(-8, 8, 1000), [0.0, -0.0, 1.0, 3.0e38]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(NO.bf16_round(a), ref)


def test_single_channel_conv_is_scipy_correlate():
    g = np.random.default_rng(1)
    x = g.standard_normal((7, 7, 7, 1))
    w = g.standard_normal((1, 27, 1))
    y = NO.conv3d(x, w)
    k = w[0, :, 0].reshape(3, 3, 3)
    ref = ndimage.correlate(x[..., 0], k, mode="constant", cval=0.0)
    assert np.allclose(y[..., 0], ref, rtol=1e-12, atol=1e-12)


def test_conv_planes_is_scipy_correlate_per_channel_pair():
    """The plane-restricted convolution (used to check single planes of large
    grids) against scipy's correlation summed over input channels."""
    g = np.random.default_rng(11)
    x = g.standard_normal((7, 7, 7, 3))
    w = g.standard_normal((2, 27, 3))
    b = g.standard_normal(2)
    zs = [0, 3, 6]
    got = NO.conv3d_planes(x, w, b, zs)
    for o in range(2):
        ref = sum(ndimage.correlate(x[..., c], w[o, :, c].reshape(3, 3, 3), mode="constant", cval=0.0)
                  for c in range(3)) + b[o]
        assert np.allclose(got[..., o], ref[zs], rtol=1e-12, atol=1e-12)


def test_dgrad_is_the_adjoint():
    g = np.random.default_rng(2)
    x = g.standard_normal((6, 6, 6, 8))
    w = g.standard_normal((16, 27, 8))
    dy = g.standard_normal((6, 6, 6, 16))
    lhs = np.sum(NO.conv3d(x, w) * dy)
    rhs = np.sum(x * NO.conv3d_dgrad(dy, w))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_wgrad_finite_differences():
    g = np.random.default_rng(3)
    x = g.standard_normal((5, 5, 5, 4))
    w = g.standard_normal((3, 27, 4))
    b = g.standard_normal(3)
    dy = g.standard_normal((5, 5, 5, 3))
    gw, gb = NO.conv3d_wgrad(x, dy)
    f = lambda ww, bb: np.sum(NO.conv3d(x, ww, bb) * dy)
    eps = 1e-6
    for (o, t, c) in [(0, 0, 0), (2, 13, 3), (1, 26, 1), (0, 7, 2)]:
        wp = w.copy(); wp[o, t, c] += eps
        wm = w.copy(); wm[o, t, c] -= eps
        assert abs((f(wp, b) - f(wm, b)) / (2 * eps) - gw[o, t, c]) < 1e-6 * (1 + abs(gw[o, t, c]))
    bp = b.copy(); bp[1] += eps
    bm = b.copy(); bm[1] -= eps
    assert abs((f(w, bp) - f(w, bm)) / (2 * eps) - gb[1]) < 1e-6 * (1 + abs(gb[1]))


def test_pool_up_adjoint():
    g = np.random.default_rng(4)
    a = g.standard_normal((8, 8, 8, 2))
    c = g.standard_normal((4, 4, 4, 2))
    # <pool(a), c> = <a, up(c)/8>
    assert abs(np.sum(NO.pool2(a) * c) - np.sum(a * NO.up2(c)) / 8) < 1e-12


# ------------------------------------------------------------------ the composed network
def _random_weights(seed, scale=1.0):
    g = np.random.default_rng(seed)
    ws, bs = [], []
    for ci, co in zip(NO.CINS, NO.COUTS):
        ws.append(scale * g.standard_normal((co, 27, ci)) / np.sqrt(27 * ci))
        bs.append(0.1 * g.standard_normal(co))
    return ws, bs


def _div_operator(n, seed):
    """A = -L of a case (b) problem (r^-4 profile in 3D, m in [2, 3.5]) from the
    FP64 oracle, zero volume constraint."""
    import oracle as O
    from paper_1905_08375_amd import fields as F
    g = np.random.default_rng(seed)
    R = 4
    P = O.Problem(dim=3, n=n, R=R, form="div", kernel="frac")
    delta = g.uniform(2.0, 3.5, (n, n, n)) / n
    coef = np.exp(g.normal(0.0, 0.5, (n, n, n)))
    apply_A = lambda z: -O.apply(P, delta, coef, F.pad(z, R))
    dinv = 1.0 / O.div_diag(P, delta, coef)
    return apply_A, dinv


def test_unet_backward_equals_finite_differences():
    """The energy-norm loss of the linear two-level preconditioner, composed
    from the layers above (13 convolutions, 3 poolings, 3 upsamplings with skip
    sums, input scaling by D^-1/2 and unit RMS, output unscaling), in exact
    FP64 on an 8^3 field: its backward pass (every layer's weight gradient)
    against central finite differences of the loss.  The network is linear and
    each weight enters it once, so the loss is quadratic in any single weight
    and the central difference is exact up to rounding."""
    n = 8
    apply_A, dinv = _div_operator(n, 3)
    g = np.random.default_rng(4)
    e = g.standard_normal((n, n, n))
    r = apply_A(e)
    ws, _ = _random_weights(5)
    ident = lambda a: a
    loss, gws = NO.energy_grads(ws, r, e, dinv, apply_A, bf=ident, bfw=ident)
    assert np.isfinite(loss) and loss > 0
    rng = np.random.default_rng(6)
    h = 1e-2
    for li in range(13):
        co_max = 1 if li == 12 else NO.COUTS[li]
        ci_max = 1 if li == 0 else NO.CINS[li]
        scale = np.abs(gws[li][:co_max, :, :ci_max]).max()
        assert scale > 0, li
        for _ in range(3):
            o, t, c = int(rng.integers(co_max)), int(rng.integers(27)), int(rng.integers(ci_max))
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[li][o, t, c] += h
            wm[li][o, t, c] -= h
            lp = NO.energy_loss(wp, r, e, dinv, apply_A, bf=ident)[0]
            lm = NO.energy_loss(wm, r, e, dinv, apply_A, bf=ident)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gws[li][o, t, c]) <= 1e-8 * scale, (li, o, t, c, fd, gws[li][o, t, c])
    # with a zero network z = D^-1 r (plain Jacobi), whose A-norm error is below that of z = 0
    assert NO.energy_loss([0 * w for w in ws], r, e, dinv, apply_A, bf=ident)[0] < 1.0


def test_activated_unet_backward_equals_finite_differences():
    """The activated network (biases, ReLU after every hidden layer) in exact
    FP64 on an 8^3 input: the backward pass of sum(dhead * head) against
    central finite differences for sampled weights and biases of each layer
    (steps small enough that no ReLU switches)."""
    g = np.random.default_rng(7)
    S = 8
    x = np.zeros((S, S, S, 8))
    x[..., :3] = g.standard_normal((S, S, S, 3))
    ws, bs = _random_weights(8)
    dhead = g.standard_normal((S, S, S, 16))
    ident = lambda a: a
    head, A = NO.unet_forward(ws, bs, x, linear=False, bf=ident)
    gws, gbs = NO.unet_backward(ws, A, dhead, linear=False, bf=ident, bfw=ident)
    f = lambda ww, bb: np.sum(NO.unet_forward(ww, bb, x, linear=False, bf=ident)[0] * dhead)
    rng = np.random.default_rng(9)
    h = 1e-6
    for li in range(13):
        ci_max = 3 if li == 0 else NO.CINS[li]
        scale = max(np.abs(gws[li]).max(), np.abs(gbs[li]).max())
        for _ in range(2):
            o, t, c = int(rng.integers(NO.COUTS[li])), int(rng.integers(27)), int(rng.integers(ci_max))
            wp = [w.copy() for w in ws]; wm = [w.copy() for w in ws]
            wp[li][o, t, c] += h; wm[li][o, t, c] -= h
            fd = (f(wp, bs) - f(wm, bs)) / (2 * h)
            assert abs(fd - gws[li][o, t, c]) <= 1e-5 * scale, (li, "w", fd, gws[li][o, t, c])
        o = int(rng.integers(NO.COUTS[li]))
        bp = [b.copy() for b in bs]; bm = [b.copy() for b in bs]
        bp[li][o] += h; bm[li][o] -= h
        fd = (f(ws, bp) - f(ws, bm)) / (2 * h)
        assert abs(fd - gbs[li][o]) <= 1e-5 * scale, (li, "b", fd, gbs[li][o])


def test_adam_step_formula():
    """The first Adam steps from zero moments: the update of each weight is
    lr * m_hat / (sqrt(v_hat) + eps), which at step 1 is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.ones(4)
    w1, m, v = NO.adam_step(w, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(w - w1, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    w2, m, v = NO.adam_step(w1, 2 * g, m, v, 2, 0.01)
    m2 = 0.9 * 0.1 * g + 0.1 * 2 * g
    v2 = 0.999 * 0.001 * g * g + 0.001 * 4 * g * g
    want = 0.01 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(w1 - w2, want, rtol=1e-12, atol=0)
