"""Training of the learned preconditioner on the GPU against the network
oracle: the energy-norm weight gradients of every layer, the Adam update,
the activated (three-input) network's forward pass, and the shipped training
recipe run from a zero output layer."""
import os
import struct
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle import net_oracle as NO
from paper_1905_08375_amd import fields as F
from paper_1905_08375_amd import ndl
from gpuhelp import say

pytestmark = pytest.mark.gpu

CINS = NO.CINS
# Adam's decay rates as the library stores them (FP32 0.9 and 0.999)
B1, B2 = float(np.float32(0.9)), float(np.float32(0.999))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def write_layers(net, layers):
    """Replace the net's FP32 weights and biases by `layers` ([cout][KP], [cout]
    pairs) through the library's file format (8-byte magic, int64 step, then
    per layer int32 (cout, KP), weights, biases) and reload it."""
    fd, path = tempfile.mkstemp(suffix=".bin")
    os.close(fd)
    try:
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
        ndl.ndl_net_load(net, path)
    finally:
        os.remove(path)


def random_bf16_layers(seed):
    """Random weights exactly representable in BF16 (so that the FP32 masters
    and the BF16 copies the kernels read agree), every layer non-zero."""
    g = np.random.default_rng(seed)
    out = []
    for li, (ci, co) in enumerate(zip(CINS, NO.COUTS)):
        w = NO.bf16_round(g.standard_normal((co, 27, ci)) / np.sqrt(27 * ci))
        out.append((NO.pack_weights(w).astype(np.float32), (0.1 * g.standard_normal(co)).astype(np.float32)))
    return out


def energy_case(n, seed):
    """An FP32 3D case (b) plan, a smooth-plus-noise error e and r = A e from
    the library's own apply (both FP32 device fields), and the oracle's view of
    the same problem: A z from the FP64 direct sum on the FP32-rounded delta and
    c, and D^-1 rounded as the library rounds it."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    plan, _, _, w = PT.problem_3d(n, seed)
    xs = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    g = np.random.default_rng(seed)
    e64 = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z) + 0.2 * g.standard_normal((n, n, n))
    e = torch.from_numpy(e64.astype(np.float32)).cuda().contiguous()
    r = PT.neg_L(plan, e, n).contiguous()
    torch.cuda.synchronize()
    R = 4
    P = O.Problem(dim=3, n=n, R=R, form="div", kernel="frac")
    d32, c32 = f32(w["delta"]), f32(w["coef"])
    apply_A = lambda z: -O.apply(P, d32, c32, F.pad(z, R))
    diag = np.abs(O.div_diag(P, d32, c32))
    dinv = (np.float32(1.0) / diag.astype(np.float32)).astype(np.float64)
    return plan, e, r, apply_A, dinv


def test_energy_gradients_and_adam_match_the_oracle():
    """One energy-norm training step (linear mode, lr = 0) at 16^3: every
    layer's weight and bias gradient against the oracle's backward pass through
    the whole U-Net (conv, pool, upsample, skip sums, the energy loss through
    the two-level z), with BF16 rounding at the GPU's storage points, to within
    twice the spread that rounding flips give the oracle itself; the loss
    against the oracle's loss.  A second step on the same data gives the same
    gradients bit for bit (fixed-order reductions), and its Adam update of
    every weight equals the formula applied to the GPU's gradient and moments."""
    import torch
    n = 16
    say(f"case energy gradients vs oracle n={n}")
    plan, e, r, apply_A, dinv = energy_case(n, 9)
    layers = random_bf16_layers(21)
    net = ndl.ndl_net_create(seed=3)
    write_layers(net, layers)
    ndl.ndl_net_set_linear(net, True)
    loss = ndl.ndl_net_train_step_energy(net, plan, r.reshape(1, n, n, n), e.reshape(1, n, n, n), 0.0)
    torch.cuda.synchronize()
    ws = [NO.unpack_weights(w.astype(np.float64), ci) for (w, _), ci in zip(layers, CINS)]
    r64, e64 = f32(r.cpu().numpy()), f32(e.cpu().numpy())
    loss_ref, st = NO.energy_loss(ws, r64, e64, dinv, apply_A, f32=f32)
    gz = 2.0 * (st["az"] - r64) / st["den"]
    dhead = np.zeros((n, n, n, 16))
    dhead[..., 0] = f32(gz * st["sq"] / (st["rscale"] * NO.TARGET_SCALE))
    gws, gbs = NO.unet_backward(ws, st["A"], dhead, linear=True)
    say(f"  loss gpu {loss:.7f} oracle {loss_ref:.7f}")
    assert abs(loss - loss_ref) <= 1e-5 * abs(loss_ref)
    # The tolerance: the GPU accumulates in FP32 in another order, so a value
    # that lies near a BF16 rounding boundary can round the other way.  Through
    # 13 layers such flips move the gradients by a fixed amount, measured here
    # on the oracle itself by perturbing every value by 1e-6 of itself before
    # each BF16 rounding (about the FP32 accumulation error); the unrounded
    # FP64 oracle shows how far the BF16 rounding points themselves move them.
    calls = [0]

    def bf_pert(a):
        calls[0] += 1
        noise = np.random.default_rng(calls[0]).standard_normal(np.shape(a))
        return NO.bf16_round(np.asarray(a) * (1.0 + 1e-6 * noise))

    _, stp = NO.energy_loss(ws, r64, e64, dinv, apply_A, bf=bf_pert, f32=f32)
    dhp = np.zeros((n, n, n, 16))
    dhp[..., 0] = f32(2.0 * (stp["az"] - r64) / stp["den"] * stp["sq"] / (stp["rscale"] * NO.TARGET_SCALE))
    gws_p, gbs_p = NO.unet_backward(ws, stp["A"], dhp, linear=True, bf=bf_pert)
    ident = lambda a: np.asarray(a, dtype=np.float64)
    _, stx = NO.energy_loss(ws, r64, e64, dinv, apply_A, bf=ident, f32=f32)
    dhx = np.zeros((n, n, n, 16))
    dhx[..., 0] = f32(2.0 * (stx["az"] - r64) / stx["den"] * stx["sq"] / (stx["rscale"] * NO.TARGET_SCALE))
    gws_x, _ = NO.unet_backward(ws, stx["A"], dhx, linear=True, bf=ident, bfw=ident)
    g1 = []
    sq_gpu = sq_exact = 0.0
    for li in range(13):
        gw = ndl.ndl_net_layer_tensor(net, li, ndl.NET_GW)
        gb = ndl.ndl_net_layer_tensor(net, li, ndl.NET_GB)
        g1.append((gw, gb))
        got = NO.unpack_weights(gw.astype(np.float64), CINS[li])
        ref = gws[li]
        nrm = np.linalg.norm(ref)
        err = np.linalg.norm(got - ref) / nrm
        errb = np.linalg.norm(gb - gbs[li]) / np.linalg.norm(gbs[li])
        spread = np.linalg.norm(gws_p[li] - ref) / nrm
        spreadb = np.linalg.norm(gbs_p[li] - gbs[li]) / np.linalg.norm(gbs[li])
        exact = np.linalg.norm(gws_x[li] - ref) / nrm
        sq_gpu += err ** 2
        sq_exact += exact ** 2
        say(f"  layer {li:2d} |g| {nrm:.3e} rel l2 {err:.2e} (flip spread {spread:.2e}, unrounded {exact:.2e})"
            f" bias {errb:.2e} (spread {spreadb:.2e})")
        assert err <= 2.0 * spread + 1e-4, (li, err, spread)
        assert errb <= 2.0 * spreadb + 1e-4, (li, errb, spreadb)
        # the padded K entries stay zero
        assert np.all(gw[:, 27 * CINS[li]:] == 0)
    # the rounding points match: over all layers the GPU sits closer to the
    # BF16-rounded oracle than the unrounded one does
    say(f"  rms over layers: gpu {np.sqrt(sq_gpu / 13):.2e}, unrounded oracle {np.sqrt(sq_exact / 13):.2e}")
    assert sq_gpu < sq_exact
    # Adam: after the lr = 0 step the weights are unchanged and the moments hold
    # (1 - b1) g and (1 - b2) g^2; a second step with lr > 0 on the same data
    mom = [(ndl.ndl_net_layer_tensor(net, li, ndl.NET_MW).astype(np.float64),
            ndl.ndl_net_layer_tensor(net, li, ndl.NET_VW).astype(np.float64)) for li in range(13)]
    for li in range(13):
        w0 = ndl.ndl_net_layer_tensor(net, li, ndl.NET_W)
        assert np.array_equal(w0, layers[li][0]), li
        g = g1[li][0].astype(np.float64)
        assert np.allclose(mom[li][0], (1.0 - B1) * g, rtol=1e-6, atol=0)
        assert np.allclose(mom[li][1], (1.0 - B2) * g * g, rtol=1e-6, atol=1e-30)
    lr = 1e-3
    ndl.ndl_net_train_step_energy(net, plan, r.reshape(1, n, n, n), e.reshape(1, n, n, n), lr)
    torch.cuda.synchronize()
    worst = 0.0
    for li in range(13):
        gw2 = ndl.ndl_net_layer_tensor(net, li, ndl.NET_GW)
        assert np.array_equal(gw2, g1[li][0]), li
        w0 = layers[li][0].astype(np.float64)
        w2 = ndl.ndl_net_layer_tensor(net, li, ndl.NET_W).astype(np.float64)
        g = g1[li][0].astype(np.float64)
        want, _, _ = NO.adam_step(w0, g, mom[li][0], mom[li][1], 2, lr, b1=B1, b2=B2)
        # FP32 arithmetic: the update to 1e-5 of lr, plus the rounding of w
        tol = 1e-5 * lr + 2.0 * np.finfo(np.float32).eps * np.abs(w0)
        assert np.all(np.abs(w2 - want) <= tol), (li, np.abs(w2 - want).max())
        worst = max(worst, np.abs((w0 - w2) - (w0 - want)).max() / lr)
    say(f"  adam step 2: worst update error / lr {worst:.2e}")


@pytest.mark.parametrize("n", [16, 32])
def test_activated_network_matches_the_oracle(n):
    """The default (activated) network on its three inputs at 16^3 and 32^3:
    r / rms(r), log c standardised over the grid, m / 4; biases and ReLU after
    every hidden layer; the inference path (skip sums formed while staging)
    against the oracle's forward pass with the GPU's initial weights rounded to
    BF16 and BF16 at the same storage points, to within twice the spread that
    rounding flips give the oracle itself and closer than the unrounded
    network."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    say(f"case activated network forward n={n}")
    plan, _, _, w = PT.problem_3d(n, 13)
    net = ndl.ndl_net_create(seed=17)
    g = np.random.default_rng(n)
    r = g.standard_normal((n, n, n)).astype(np.float32)
    z = torch.empty((n, n, n), device="cuda")
    ndl.ndl_precond_apply(net, plan, torch.from_numpy(r).cuda(), z)
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.float64)
    ws = [NO.bf16_round(NO.unpack_weights(ndl.ndl_net_layer_tensor(net, li, ndl.NET_W).astype(np.float64), CINS[li]))
          for li in range(13)]
    bs = [ndl.ndl_net_layer_tensor(net, li, ndl.NET_B).astype(np.float64) for li in range(13)]
    r64 = r.astype(np.float64)
    rscale = np.sqrt(r64.size / np.sum(r64 * r64))
    lc = np.log(f32(w["coef"]))
    mu = lc.mean()
    var = np.mean(lc * lc) - mu * mu
    x = np.zeros((n, n, n, 8))
    x[..., 0] = NO.bf16_round(f32(r64 * rscale))
    x[..., 1] = NO.bf16_round(f32((lc - mu) / np.sqrt(var)))
    x[..., 2] = NO.bf16_round(f32(f32(w["delta"]) * n * 0.25))
    scale = rscale * NO.TARGET_SCALE
    ref = NO.unet_forward(ws, bs, x, linear=False)[0][..., 0] / scale
    # the spread that rounding flips give the oracle itself (every value moved
    # by 1e-6 of itself before each BF16 rounding), and the unrounded network
    calls = [0]

    def bf_pert(a):
        calls[0] += 1
        noise = np.random.default_rng(calls[0]).standard_normal(np.shape(a))
        return NO.bf16_round(np.asarray(a) * (1.0 + 1e-6 * noise))

    nrm = np.linalg.norm(ref)
    spread = np.linalg.norm(NO.unet_forward(ws, bs, x, linear=False, bf=bf_pert)[0][..., 0] / scale - ref) / nrm
    exact = np.linalg.norm(NO.unet_forward(ws, bs, x, linear=False, bf=lambda a: a)[0][..., 0] / scale - ref) / nrm
    err = np.linalg.norm(got - ref) / nrm
    say(f"  rel l2 {err:.2e} (flip spread {spread:.2e}, unrounded {exact:.2e})")
    assert np.isfinite(got).all()
    assert err <= 2.0 * spread + 1e-5
    assert err < exact


def test_training_recipe_from_a_zero_output_layer_gains_over_jacobi():
    """The shipped recipe (pairs from warm-started plain-CG runs, energy-norm
    training of the linear network from a zero output layer, i.e. from plain
    Jacobi) run on the GPU at 64^3 for 300 steps on 4 training fields, then
    flexible PCG on a held-out field against plain Jacobi-CG: fewer iterations,
    with both final residuals recomputed by the FP64 oracle over every node."""
    import torch
    from paper_1905_08375_amd import precond_train as PT
    n = 64
    say(f"case training recipe n={n}")
    data = PT.make_pairs(n, range(4), ks=(4, 8, 16, 32, 48, 64, 96), log=say)
    net = PT.new_net(seed=1)
    hist = PT.train(net, data, steps=300, lr=1e-3, log=say)
    assert all(np.isfinite(hist))
    assert np.mean(hist[-20:]) < np.mean(hist[:5])
    seed = 100
    plan, b, _, w = PT.problem_3d(n, seed)
    xp = torch.zeros_like(b)
    rc, rep = ndl.ndl_cg_solve([plan], [b], [xp], rtol=1e-8, max_iter=20000)
    xl = torch.zeros_like(b)
    rc2, rep2 = ndl.ndl_cg_solve([plan], [b], [xl], rtol=1e-8, precond=1, net=net, max_iter=20000)
    torch.cuda.synchronize()
    say(f"  plain {rep[0].iters} it, learned {rep2[0].iters} it (fell back {rep2[0].fell_back})")
    assert rc == 0 and rc2 == 0 and not rep2[0].fell_back
    assert rep2[0].iters <= 0.7 * rep[0].iters
    R = 4
    P = O.Problem(dim=3, n=n, R=R, form="div", kernel="frac")
    d32, c32 = f32(w["delta"]), f32(w["coef"])
    bb = b.cpu().numpy()
    for x in (xp, xl):
        res = bb + O.apply(P, d32, c32, F.pad(x.cpu().numpy(), R))
        rel = np.linalg.norm(res) / np.linalg.norm(bb)
        say(f"  oracle residual {rel:.3e}")
        assert rel <= 1.05e-8
