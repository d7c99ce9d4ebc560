"""Network kernels (BF16 MFMA forward/data gradient, FP32 weight gradient) against
the FP64 numpy reference with the same BF16 rounding points."""
import numpy as np
import pytest

from oracle import net_oracle as NO
from paper_1905_08375_amd import ndl
from gpuhelp import say

pytestmark = pytest.mark.gpu

PAIRS = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 16)]


@pytest.mark.parametrize("cin,cout", PAIRS)
@pytest.mark.parametrize("S", [16, 20])
def test_conv_layer(cin, cout, S):
    import torch
    say(f"case conv {cin}->{cout} S={S}")
    g = np.random.default_rng(cin * 100 + cout + S)
    x = NO.bf16_round(g.standard_normal((S, S, S, cin)))
    w = g.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin)
    b = g.standard_normal(cout)
    dy = g.standard_normal((S, S, S, cout))
    wk = NO.pack_weights(w)
    d = lambda a, t=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(t).cuda()
    xb = torch.from_numpy(NO.bf16_bits(x).view(np.int16)).cuda()
    y = torch.zeros((S, S, S, cout), device="cuda")
    dx = torch.zeros((S, S, S, cin), device="cuda")
    gw = torch.zeros(wk.shape, device="cuda")
    gb = torch.zeros(cout, device="cuda")
    # the input layer (8 channels) needs no data gradient and has none
    ndl.ndl_net_conv_test(cin, cout, S, xb, d(wk), d(b), y=y, dy=d(dy), dx=dx if cin >= 16 else None, gw=gw, gb=gb)
    torch.cuda.synchronize()
    wr = NO.bf16_round(w)
    yref = NO.conv3d(x, wr, b)
    err = np.abs(y.cpu().numpy() - yref).max() / np.abs(yref).max()
    say("  fwd", err)
    assert err < 1e-5
    if cin >= 16:
        dxref = NO.conv3d_dgrad(NO.bf16_round(dy), wr)
        err = np.abs(dx.cpu().numpy() - dxref).max() / np.abs(dxref).max()
        say("  dgrad", err)
        assert err < 1e-5
    gwref, gbref = NO.conv3d_wgrad(x, dy.astype(np.float32).astype(np.float64))
    got = NO.unpack_weights(gw.cpu().numpy().astype(np.float64), cin)
    err = np.abs(got - gwref).max() / np.abs(gwref).max()
    say("  wgrad", err)
    assert err < 1e-5
    assert np.abs(gb.cpu().numpy() - gbref).max() <= 1e-5 * np.abs(gbref).max()
    # padded K entries of the weight gradient stay zero
    assert np.all(gw.cpu().numpy()[:, 27 * cin:] == 0)


def test_train_step_reduces_loss_and_roundtrips(tmp_path):
    import torch
    say("case train")
    net = ndl.ndl_net_create(seed=7)
    assert ndl.ndl_net_num_params(net) > 1e5
    s, B = 32, 2
    g = np.random.default_rng(5)
    e = torch.from_numpy(np.cumsum(np.cumsum(g.standard_normal((B, s, s, s)), axis=1), axis=2).astype(np.float32)).cuda()
    e /= e.std()
    r = torch.from_numpy(g.standard_normal((B, s, s, s)).astype(np.float32)).cuda()
    feat = torch.zeros((B, 2, s, s, s), device="cuda")
    losses = [ndl.ndl_net_train_step(net, r, feat, e, 1e-3) for _ in range(25)]
    say("  losses", losses[0], losses[-1])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0]
    p = str(tmp_path / "w.bin")
    ndl.ndl_net_save(net, p)
    net2 = ndl.ndl_net_create(seed=99)
    ndl.ndl_net_load(net2, p)
    l1 = ndl.ndl_net_train_step(net, r, feat, e, 0.0)
    l2 = ndl.ndl_net_train_step(net2, r, feat, e, 0.0)
    assert abs(l1 - l2) <= 1e-6 * abs(l1)
