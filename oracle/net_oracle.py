"""FP64 numpy reference of the preconditioner network's layers (TEST INFRASTRUCTURE).

Layout NDHWC ([S][S][S][C]); 3x3x3 convolution with zero padding; weights
[C_out][27][C_in] with tap = (dz*3 + dy)*3 + dx, offsets d - 1.  BF16 rounding
(round to nearest even) is applied where the GPU path stores BF16, so that the
comparison isolates the accumulation order.
"""
import numpy as np


def bf16_round(a):
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    out = ((u + r) >> 16).astype(np.uint32) << 16
    special = (u & 0x7F800000) == 0x7F800000
    out = np.where(special, (u >> 16 << 16).astype(np.uint32), out.astype(np.uint32))
    return out.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(a):
    f = np.asarray(bf16_round(a), dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


TAPS = [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]


def _shift(x, dz, dy, dx):
    """x[z + dz - 1, y + dy - 1, x + dx - 1] with zero outside."""
    S = x.shape[0]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[dz:dz + S, dy:dy + S, dx:dx + S]


def conv3d(x, w, b=None):
    """y[v][o] = b[o] + sum_{tap, c} w[o][tap][c] x[v + off(tap)][c]."""
    S = x.shape[0]
    y = np.zeros((S, S, S, w.shape[0]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += np.einsum("zyxc,oc->zyxo", _shift(x, dz, dy, dx), w[:, t, :])
    if b is not None:
        y += b
    return y


def conv3d_planes(x, w, b, zs):
    """The planes z in zs of conv3d(x, w, b), each from its own three input planes."""
    S = x.shape[0]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = []
    for z in zs:
        y = np.zeros((S, S, w.shape[0]))
        for t, (dz, dy, dx) in enumerate(TAPS):
            y += p[z + dz, dy:dy + S, dx:dx + S] @ w[:, t, :].T
        if b is not None:
            y += b
        out.append(y)
    return np.stack(out)


def conv3d_dgrad(dy, w):
    """dx[v][c] = sum_{tap, o} w[o][tap][c] dy[v - off(tap)][o] (the adjoint of conv3d)."""
    S = dy.shape[0]
    dx_ = np.zeros((S, S, S, w.shape[2]))
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        dx_ += np.einsum("zyxo,oc->zyxc", _shift(dy, 2 - dz, 2 - dyy, 2 - dxx), w[:, t, :])
    return dx_


def conv3d_wgrad(x, dy):
    """gw[o][tap][c] = sum_v dy[v][o] x[v + off(tap)][c], gb[o] = sum_v dy[v][o]."""
    gw = np.zeros((dy.shape[3], 27, x.shape[3]))
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        gw[:, t, :] = np.einsum("zyxo,zyxc->oc", dy, _shift(x, dz, dyy, dxx))
    return gw, dy.sum(axis=(0, 1, 2))


def pool2(x):
    S = x.shape[0] // 2
    return x.reshape(S, 2, S, 2, S, 2, -1).mean(axis=(1, 3, 5))


def up2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def pack_weights(w):
    """[C_out][27][C_in] -> [C_out][K] with K = 27 C_in rounded up to 32 (k = tap C_in + c)."""
    co, _, ci = w.shape
    K = ((27 * ci + 31) // 32) * 32
    out = np.zeros((co, K))
    out[:, :27 * ci] = w.reshape(co, 27 * ci)
    return out


def unpack_weights(wk, cin):
    co = wk.shape[0]
    return wk[:, :27 * cin].reshape(co, 27, cin)


# ------------------------------------------------------------------ the whole network
# The preconditioner network: a 4-level U-Net of 3x3x3 convolutions.  Level l
# works on a cube of side S / 2^l.  Layer order, input and output channels:
#   0: 8->16, 1: 16->16            (level 0, encoder)
#   2: 16->16, 3: 16->16           (level 1, input = pool2 of layer 1)
#   4: 16->32, 5: 32->32           (level 2, input = pool2 of layer 3)
#   6: 32->32, 7: 32->32           (level 3, input = pool2 of layer 5)
#   8: 32->32, 9: 32->16           (level 2, input = up2(layer 7) + layer 5)
#   10: 16->16                     (level 1, input = up2(layer 9) + layer 3)
#   11: 16->16                     (level 0, input = up2(layer 10) + layer 1)
#   12: 16->16 output layer, linear, FP32, channel 0 used
# Hidden layers apply ReLU after the bias unless the network is linear (no
# biases, no activations).  `bf` is applied wherever an activation is stored
# (BF16 on the GPU); pass the identity for an exact FP64 network.
CINS = [8, 16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16]
COUTS = [16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16, 16]


def _ident(a):
    return a


def unet_forward(ws, bs, x, linear=True, bf=bf16_round):
    """ws[i]: [C_out][27][C_in] weights, bs[i]: [C_out] biases (ignored when
    linear), x: [S][S][S][8] input.  Returns (head, acts) with head the FP32
    output [S][S][S][16] and acts the dict of every stored activation, which
    the backward pass reads."""
    A = {"x": x}

    def conv(i, a):
        y = conv3d(a, ws[i], None if linear else bs[i])
        if i == 12:
            return y
        if not linear:
            y = np.maximum(y, 0.0)
        return bf(y)

    A[0] = conv(0, x)
    A[1] = conv(1, A[0])
    A["p1"] = bf(pool2(A[1]))
    A[2] = conv(2, A["p1"])
    A[3] = conv(3, A[2])
    A["p2"] = bf(pool2(A[3]))
    A[4] = conv(4, A["p2"])
    A[5] = conv(5, A[4])
    A["p3"] = bf(pool2(A[5]))
    A[6] = conv(6, A["p3"])
    A[7] = conv(7, A[6])
    A["u2"] = bf(up2(A[7]) + A[5])
    A[8] = conv(8, A["u2"])
    A[9] = conv(9, A[8])
    A["u1"] = bf(up2(A[9]) + A[3])
    A[10] = conv(10, A["u1"])
    A["u0"] = bf(up2(A[10]) + A[1])
    A[11] = conv(11, A["u0"])
    head = conv(12, A[11])
    return head, A


LAYER_INPUT = {0: "x", 1: 0, 2: "p1", 3: 2, 4: "p2", 5: 4, 6: "p3", 7: 6, 8: "u2", 9: 8, 10: "u1", 11: "u0",
               12: 11}


def up2_adjoint(d):
    """Adjoint of up2: each coarse voxel collects the sum of its 8 children."""
    S = d.shape[0] // 2
    return d.reshape(S, 2, S, 2, S, 2, -1).sum(axis=(1, 3, 5))


def unet_backward(ws, A, dhead, linear=True, bf=bf16_round, bfw=bf16_round):
    """Gradients of sum(dhead * head) with respect to every weight and bias,
    by the chain rule through unet_forward's graph.  The data gradient of a
    convolution reads bf(dY) and the weights bfw(w) (the GPU's BF16 operands);
    the weight gradient reads the stored layer input and the FP32 dY.
    Returns (gws, gbs) lists indexed by layer."""
    gws, gbs = [None] * 13, [None] * 13
    d = {12: dhead}

    def back(i):
        dy = d[i]
        if i != 12 and not linear:
            dy = np.where(A[i] > 0.0, dy, 0.0)  # ReLU mask on the stored output
        gws[i], gbs[i] = conv3d_wgrad(A[LAYER_INPUT[i]], dy)
        if i == 0:
            return None
        return conv3d_dgrad(bf(dy), bfw(ws[i]))

    d[11] = back(12)
    du0 = back(11)
    d[10] = up2_adjoint(du0)
    d1_skip = du0
    du1 = back(10)
    d[9] = up2_adjoint(du1)
    d3_skip = du1
    d[8] = back(9)
    du2 = back(8)
    d[7] = up2_adjoint(du2)
    d5_skip = du2
    d[6] = back(7)
    dp3 = back(6)
    d[5] = d5_skip + up2(dp3) / 8.0
    d[4] = back(5)
    dp2 = back(4)
    d[3] = d3_skip + up2(dp2) / 8.0
    d[2] = back(3)
    dp1 = back(2)
    d[1] = d1_skip + up2(dp1) / 8.0
    d[0] = back(1)
    back(0)
    return gws, gbs


# ------------------------------------------------------------------ energy-norm training loss
# The two-level preconditioner of linear mode: with D the diagonal of A = -L,
#   rs = r D^-1/2,  rscale = sqrt(N / sum rs^2),  x[..., 0] = rs * rscale,
#   z = D^-1 r + D^-1/2 head[..., 0] / (rscale * T),
# and the loss for a pair (r, e) with A e = r is the A-norm error
#   loss = ||e - z||_A^2 / ||e||_A^2 = (e - z).(r - A z) / (e.r).
TARGET_SCALE = 32.0


def energy_loss(ws, r, e, dinv, apply_A, bf=bf16_round, f32=None):
    """Loss and the intermediate fields of the linear-mode energy loss.
    apply_A(z) returns A z on the grid.  f32 rounds where the GPU stores FP32
    (identity by default)."""
    f32 = f32 or _ident
    S = r.shape[0]
    sq = np.sqrt(dinv)
    rs = f32(r * sq)
    rscale = np.sqrt(rs.size / np.sum(rs * rs))
    x = np.zeros((S, S, S, 8))
    x[..., 0] = bf(rs * rscale)
    head, A = unet_forward(ws, None, x, linear=True, bf=bf)
    y = f32(head[..., 0])
    z = f32(r * dinv + sq * y / (rscale * TARGET_SCALE))
    az = apply_A(z)
    den = np.sum(e * r)
    loss = np.sum((e - z) * (r - az)) / den
    return loss, dict(A=A, z=z, az=az, den=den, sq=sq, rscale=rscale)


def energy_grads(ws, r, e, dinv, apply_A, bf=bf16_round, bfw=bf16_round, f32=None):
    """Loss and the weight gradients of energy_loss (A symmetric): the loss
    gradient with respect to z is 2 (A z - r) / (e.r), carried to the output
    layer through z's dependence on channel 0 of the head."""
    f32 = f32 or _ident
    loss, st = energy_loss(ws, r, e, dinv, apply_A, bf=bf, f32=f32)
    gz = 2.0 * (st["az"] - r) / st["den"]
    dhead = np.zeros(r.shape + (16,))
    dhead[..., 0] = f32(gz * st["sq"] / (st["rscale"] * TARGET_SCALE))
    gws, _ = unet_backward(ws, st["A"], dhead, linear=True, bf=bf, bfw=bfw)
    return loss, gws


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction (Kingma & Ba): returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    c1 = 1.0 - b1 ** step
    c2 = 1.0 - b2 ** step
    return w - lr * (m / c1) / (np.sqrt(v / c2) + eps), m, v
