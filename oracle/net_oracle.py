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
