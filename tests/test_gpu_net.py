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


@pytest.mark.parametrize("cin,cout,S", [(8, 16, 72), (16, 16, 72), (16, 32, 72), (32, 32, 40), (32, 16, 72)])
def test_conv_layer_many_patches(cin, cout, S):
    """Forward and data gradient over many (x, y, z) patches with ragged
    edges on every axis (the patch grid is walked in its XCD order)."""
    import torch
    say(f"case conv {cin}->{cout} S={S} (many patches)")
    g = np.random.default_rng(cin * 1000 + cout + S)
    x = NO.bf16_round(g.standard_normal((S, S, S, cin)))
    w = g.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin)
    b = g.standard_normal(cout)
    dy = g.standard_normal((S, S, S, cout))
    wk = NO.pack_weights(w)
    d = lambda a, t=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(t).cuda()
    xb = torch.from_numpy(NO.bf16_bits(x).view(np.int16)).cuda()
    y = torch.zeros((S, S, S, cout), device="cuda")
    dx = torch.zeros((S, S, S, cin), device="cuda")
    ndl.ndl_net_conv_test(cin, cout, S, xb, d(wk), d(b), y=y, dy=d(dy) if cin >= 16 else None,
                          dx=dx if cin >= 16 else None)
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


@pytest.mark.parametrize("cin,cout", [(8, 16), (16, 16)])
def test_conv_layer_full_resolution_patches(cin, cout):
    """The full-resolution patch shape (8-row patches of 16 planes, weights
    in LDS) on a 130^3 grid, ragged on every axis: output planes at both
    boundaries, at patch seams and inside, against the FP64 reference."""
    import torch
    S = 130
    say(f"case conv {cin}->{cout} S={S} (full-resolution patches)")
    g = np.random.default_rng(cin * 7 + cout)
    x = NO.bf16_round(g.standard_normal((S, S, S, cin)))
    w = g.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin)
    b = g.standard_normal(cout)
    wk = NO.pack_weights(w)
    d = lambda a, t=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(t).cuda()
    xb = torch.from_numpy(NO.bf16_bits(x).view(np.int16)).cuda()
    y = torch.zeros((S, S, S, cout), device="cuda")
    ndl.ndl_net_conv_test(cin, cout, S, xb, d(wk), d(b), y=y)
    torch.cuda.synchronize()
    zs = [0, 1, 15, 16, 17, 64, 127, 128, 129]
    yref = NO.conv3d_planes(x, NO.bf16_round(w), b, zs)
    got = y.cpu().numpy()[zs]
    err = np.abs(got - yref).max() / np.abs(yref).max()
    say("  fwd", err)
    assert err < 1e-5


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


def _read_layers(net):
    """FP32 master weights and biases of each layer, read back through the
    library's save format (8-byte magic, int64 step, then per layer int32
    (cout, KP), weights [cout][KP], biases [cout])."""
    import os
    import struct
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".bin")
    os.close(fd)
    try:
        ndl.ndl_net_save(net, path)
        raw = open(path, "rb").read()
    finally:
        os.remove(path)
    off, layers = 16, []
    while off < len(raw):
        cout, kp = struct.unpack_from("<ii", raw, off)
        w = np.frombuffer(raw, np.float32, cout * kp, off + 8).reshape(cout, kp).astype(np.float64)
        b = np.frombuffer(raw, np.float32, cout, off + 8 + 4 * cout * kp).astype(np.float64)
        layers.append((w, b))
        off += 8 + 4 * (cout * kp + cout)
    return layers


@pytest.mark.parametrize("n", [8, 16, 64])
def test_linear_network_forward_matches_oracle(n):
    """The whole preconditioner network in linear mode (the shipped weights) on an
    8^3 (coarsest level 1^3), a 16^3 and a 64^3 field (every patch shape below
    the full-resolution one, the single-channel input layer and the skip sums
    formed while staging included) against the FP64 reference
    composed from the oracle's layers:
    residual scaled by D^-1/2 (D from the oracle's case (b) diagonal) and
    normalised to unit RMS, 13 convolutions without biases or activations,
    3 average poolings, 3 nearest upsamplings with skip additions, BF16 at the
    GPU's storage points, channel 0 of the output layer rescaled."""
    import torch
    import oracle as O
    from paper_1905_08375_amd import precond_train as PT
    if not __import__("os").path.exists(PT.WEIGHTS):
        pytest.skip("no trained weights in the tree")
    say(f"case linear network forward n={n}")
    plan, b, feat, w = PT.problem_3d(n, 7)
    net = PT.load_net(PT.WEIGHTS)
    g = np.random.default_rng(5)
    r = g.standard_normal((n, n, n)).astype(np.float32)
    z = torch.empty((n, n, n), device="cuda")
    ndl.ndl_precond_apply(net, plan, torch.from_numpy(r).cuda(), z)
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.float64)
    # reference
    P = O.Problem(dim=3, n=n, R=4, form="div", kernel="frac")
    diag = O.div_diag(P, w["delta"].astype(np.float32), w["coef"].astype(np.float32))
    diag = np.abs(diag)
    dinv = (np.float32(1.0) / diag.astype(np.float32)).astype(np.float64)
    sq = np.sqrt(dinv)
    rs = (r.astype(np.float64) * sq).astype(np.float32).astype(np.float64)
    rscale = np.sqrt(rs.size / np.sum(rs * rs))
    x = np.zeros((n, n, n, 8))
    x[..., 0] = NO.bf16_round(rs * rscale)
    layers = _read_layers(net)
    cins = [8, 16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16]

    def conv(i, a):
        wk, _ = layers[i]
        return NO.conv3d(a, NO.unpack_weights(NO.bf16_round(wk), cins[i]))

    bf = NO.bf16_round
    a0 = bf(conv(0, x)); a1 = bf(conv(1, a0))
    a2 = bf(conv(2, bf(NO.pool2(a1)))); a3 = bf(conv(3, a2))
    a4 = bf(conv(4, bf(NO.pool2(a3)))); a5 = bf(conv(5, a4))
    a6 = bf(conv(6, bf(NO.pool2(a5)))); a7 = bf(conv(7, a6))
    a8 = bf(conv(8, bf(NO.up2(a7) + a5))); a9 = bf(conv(9, a8))
    a10 = bf(conv(10, bf(NO.up2(a9) + a3)))
    a11 = bf(conv(11, bf(NO.up2(a10) + a1)))
    head = conv(12, a11)[..., 0]
    ref = sq * head / (rscale * PT.TARGET_SCALE)
    assert np.isfinite(got).all(), int((~np.isfinite(got)).sum())
    assert np.isfinite(ref).all(), int((~np.isfinite(ref)).sum())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say("  rel l2", err)
    assert err < 2e-3


def _write_layers(net, layers, path):
    """Save the net, replace its FP32 weights and biases by `layers`, write to path."""
    import struct
    ndl.ndl_net_save(net, path)
    raw = bytearray(open(path, "rb").read())
    off, i = 16, 0
    while off < len(raw):
        cout, kp = struct.unpack_from("<ii", raw, off)
        w, b = layers[i]
        raw[off + 8:off + 8 + 4 * cout * kp] = np.asarray(w, np.float32).tobytes()
        raw[off + 8 + 4 * cout * kp:off + 8 + 4 * (cout * kp + cout)] = np.asarray(b, np.float32).tobytes()
        off += 8 + 4 * (cout * kp + cout)
        i += 1
    open(path, "wb").write(bytes(raw))


def test_energy_training_step_follows_the_loss_gradient(tmp_path):
    """One Adam step of the energy-norm training (linear mode) moves each
    weight by lr sign(g); the sign of g is checked against central finite
    differences of the loss the same entry point reports (the loss is
    quadratic in any one weight, so the difference quotient is exact up to
    rounding), on weights of the input, encoder, decoder and output layers."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    say("case energy training gradient signs")
    n = 16
    plan, b, feat, w = PT.problem_3d(n, 9)
    # a smooth error (the part Jacobi-CG leaves, which the network targets)
    xs = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    e64 = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z) + 0.3 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    e = torch.from_numpy(e64.astype(np.float32)).cuda().reshape(1, n, n, n).contiguous()
    r = PT.neg_L(plan, e[0], n).reshape(1, n, n, n).contiguous()
    base = ndl.ndl_net_create(seed=3)
    ndl.ndl_net_set_linear(base, True)
    layers = _read_layers(base)
    path = str(tmp_path / "w.bin")

    def loss_at(lay, lr=0.0):
        _write_layers(base, lay, path)
        net = ndl.ndl_net_create(seed=3)
        ndl.ndl_net_load(net, path)
        ndl.ndl_net_set_linear(net, True)
        out = ndl.ndl_net_train_step_energy(net, plan, r, e, lr)
        torch.cuda.synchronize()
        return out, net

    lr = 1e-4
    _, stepped = loss_at(layers, lr)
    after = _read_layers(stepped)
    rng = np.random.default_rng(0)
    cins = [8, 16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16]
    checked = 0
    for li in (0, 1, 8, 10, 11, 12):
        wl = layers[li][0]
        cout = wl.shape[0]
        picks = [(int(rng.integers(cout if li != 12 else 1)), int(rng.integers(27 * (1 if li == 0 else cins[li]))))
                 for _ in range(6)]
        for co, k in picks:
            if li == 0:
                k = k * 8  # channel 0 of the input layer (the residual)
            # a perturbation several times the weight: the central difference
            # of a quadratic is exact for any h, and a large h lifts the change
            # of the loss above the BF16 rounding of the activations
            h = 0.5
            lp = [(a.copy(), bb.copy()) for a, bb in layers]
            lm = [(a.copy(), bb.copy()) for a, bb in layers]
            lp[li][0][co, k] += h
            lm[li][0][co, k] -= h
            gfd = (loss_at(lp)[0] - loss_at(lm)[0]) / (2 * h)
            step = wl[co, k] - after[li][0][co, k]
            say(f"  layer {li} w[{co}][{k}] fd {gfd:.3e} step {step:.3e}")
            if abs(gfd) < 3e-4:
                continue
            assert np.sign(step) == np.sign(gfd), (li, co, k, gfd, step)
            assert abs(abs(step) - lr) <= 0.05 * lr
            checked += 1
    assert checked >= 10


def test_fused_inference_matches_the_training_forward():
    """At 128^3 (the full-resolution patch shapes) the inference path, which
    stages the input layer from the scaled FP32 residual and forms the skip
    sums while staging, against the training forward, which stores every layer
    input: the energy loss that ndl_net_train_step_energy reports (lr = 0, so
    the weights stay) equals the same loss formed here from ndl_precond_apply,
    the Jacobi term from the oracle's diagonal and the operator's apply."""
    import torch
    import oracle as O
    from paper_1905_08375_amd import precond_train as PT
    if not __import__("os").path.exists(PT.WEIGHTS):
        pytest.skip("no trained weights in the tree")
    say("case fused inference vs training forward n=128")
    n = 128
    plan, b, feat, w = PT.problem_3d(n, 11)
    net = PT.load_net(PT.WEIGHTS)
    xs = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    g = np.random.default_rng(2)
    e64 = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z) + 0.1 * g.standard_normal((n, n, n))
    e = torch.from_numpy(e64.astype(np.float32)).cuda().contiguous()
    r = PT.neg_L(plan, e, n).contiguous()
    loss_train = ndl.ndl_net_train_step_energy(net, plan, r.reshape(1, n, n, n), e.reshape(1, n, n, n), 0.0)
    zn = torch.empty_like(r)
    ndl.ndl_precond_apply(net, plan, r, zn)
    torch.cuda.synchronize()
    P = O.Problem(dim=3, n=n, R=4, form="div", kernel="frac")
    diag = np.abs(O.div_diag(P, w["delta"].astype(np.float32), w["coef"].astype(np.float32)))
    dinv = torch.from_numpy((np.float32(1.0) / diag.astype(np.float32)).astype(np.float32)).cuda()
    z = r * dinv + zn
    az = PT.neg_L(plan, z, n)
    ed, zd, rd, ad = (t.double() for t in (e, z, r, az))
    loss_inf = float(((ed - zd) * (rd - ad)).sum() / (ed * rd).sum())
    say("  train", loss_train, "inference", loss_inf)
    assert abs(loss_inf - loss_train) <= 1e-4 * abs(loss_train)
