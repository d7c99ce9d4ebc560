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
