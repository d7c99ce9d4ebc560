"""Training and evaluation of the learned preconditioner (3D case (b) workload).

Training pairs come from plain Jacobi-CG runs of the library on seeded fields:
for each training field the solver is run to a tight tolerance (x*) and, in
one warm-started run, to k_1 < k_2 < ... iterations (x_k); the pair is the
residual r_k = b + L x_k and the correction e_k = x* - x_k on the whole
field.  The network is trained on full fields with the energy norm that CG
minimises: for the two-level preconditioner z = D^-1 r + M(r) the loss is
||e - z||_A^2 / ||e||_A^2 (A = -L), evaluated with the library's operator.

The network runs in its linear mode, M(r) = D^-1/2 N(D^-1/2 r) with N
free of activations and biases: the correction CG needs is A^-1 r, a linear
map of r, and a linear network fits it from few pairs and holds on unseen
fields, where the activated network with (r, log c, m) inputs did not.  Its
output layer starts at zero, so training starts from plain Jacobi (loss
about 1) and only moves where the energy decreases.

Every arithmetic step runs in libndl (the operator, the solves, the
network's forward/backward and Adam); torch only holds the tensors.

`python -m paper_1905_08375_amd.precond_train` writes the shipped weights
(`weights/precond_3d.bin`, linear mode).
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import fields as F
from . import ndl

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "precond_3d.bin")
TARGET_SCALE = 32.0  # the network's output scale (libndl divides its output by it)


def problem_3d(n: int, seed: int, prec=ndl.NDL_F32C, R: int = 4):
    import torch
    w = F.diffusion_3d(n=n, seed_field=seed)
    npt = np.float64 if prec == ndl.NDL_F64 else np.float32
    d = torch.from_numpy(w["delta"].astype(npt)).cuda()
    c = torch.from_numpy(w["coef"].astype(npt)).cuda()
    plan = ndl.ndl_plan_create(ndl.make_problem(3, n, R, d, c, form=ndl.NDL_DIV, prec=prec), keep=(d, c))
    b = torch.from_numpy(w["b"]).cuda()
    lc = np.log(w["coef"].astype(npt).astype(np.float64))
    feat = np.stack([(lc - lc.mean()) / lc.std(), w["delta"].astype(npt).astype(np.float64) * n / 4.0])
    return plan, b, feat, w


def neg_L(plan, x, n, R=4):
    """-L x with a zero collar (the solve operator), through ndl_apply (FP32 path)."""
    import torch
    pad = torch.zeros((n + 2 * R,) * 3, dtype=torch.float32, device="cuda")
    pad[R:R + n, R:R + n, R:R + n] = x.float()
    out = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    ndl.ndl_apply(plan, pad, out, 1)
    return -out


def cg_iterate(plan, b, iters, rtol=1e-10, x0=None):
    """Plain Jacobi-CG for `iters` iterations from x0 (zero by default)."""
    import torch
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    ndl.ndl_cg_solve([plan], [b], [x], rtol=rtol, max_iter=iters)
    return x


def make_pairs(n=256, seeds=range(8), ks=(8, 16, 32, 64, 128, 256), log=print):
    """Per training field: its plan and residual/correction pairs (r_k, e_k =
    x* - x_k) as FP32 fields, with x_k the plain-CG iterates at the iteration
    counts ks (one warm-started run per field: each segment continues from
    the previous iterate) and x* the solve to 1e-9."""
    import torch
    out = []
    for sd in seeds:
        t0 = time.perf_counter()
        plan, b, feat, _ = problem_3d(n, sd)
        xs = cg_iterate(plan, b, 100000, rtol=1e-9)
        pairs = []
        xk, done = None, 0
        for k in sorted(ks):
            xk = cg_iterate(plan, b, k - done, x0=xk)
            done = k
            ek = (xs - xk).float()
            rk = (b - neg_L(plan, xk, n)).float()
            pairs.append((rk, ek))
        out.append((plan, pairs))
        log(f"pairs: seed {sd} done in {time.perf_counter() - t0:.1f}s")
    return out


def zero_output_layer(net):
    """Zero the output layer's weights and bias (a save / edit / load round
    trip: the file is an 8-byte magic, an int64 step count, then per layer an
    int32 pair (cout, KP), FP32 weights [cout][KP] and FP32 biases [cout])."""
    import struct
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".bin")
    os.close(fd)
    try:
        ndl.ndl_net_save(net, path)
        with open(path, "rb") as f:
            raw = bytearray(f.read())
        off, last = 16, None
        while off < len(raw):
            cout, kp = struct.unpack_from("<ii", raw, off)
            last = (off, cout, kp)
            off += 8 + 4 * (cout * kp + cout)
        o, cout, kp = last
        raw[o + 8:o + 8 + 4 * (cout * kp + cout)] = bytes(4 * (cout * kp + cout))
        with open(path, "wb") as f:
            f.write(raw)
        ndl.ndl_net_load(net, path)
    finally:
        os.remove(path)


def new_net(seed=1):
    """The shipped configuration: linear mode, output layer at zero."""
    net = ndl.ndl_net_create(seed=seed)
    zero_output_layer(net)
    ndl.ndl_net_set_linear(net, True)
    return net


def load_net(path=WEIGHTS):
    net = ndl.ndl_net_create(seed=1)
    ndl.ndl_net_load(net, path)
    ndl.ndl_net_set_linear(net, True)
    return net


def train(net, data, steps=300, batch=2, lr=1e-3, steps_per_field=10, seed=0, log=print):
    """Energy-norm training (||e - z||_A / ||e||_A with z = D^-1 r + M(r)) on full fields."""
    import torch
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(steps):
        plan, pairs = data[(it // steps_per_field) % len(data)]
        pick = rng.choice(len(pairs), size=min(batch, len(pairs)), replace=False)
        r = torch.stack([pairs[i][0] for i in pick]).contiguous()
        e = torch.stack([pairs[i][1] for i in pick]).contiguous()
        lr_t = lr * (0.1 ** (it / max(steps, 1)))
        loss = ndl.ndl_net_train_step_energy(net, plan, r, e, lr_t)
        hist.append(loss)
        if it % 25 == 0 or it == steps - 1:
            log(f"train step {it} energy-loss {loss:.4f}")
    return hist


def compare(net, n=256, seed=100, rtol=1e-8, max_iter=None):
    """Plain Jacobi-CG vs learned flexible PCG on one held-out field (same outer loop)."""
    import torch
    plan, b, _, _ = problem_3d(n, seed)
    x0 = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mi = max_iter or 200000
    rc, rep = ndl.ndl_cg_solve([plan], [b], [x0], rtol=rtol, max_iter=mi)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    x1 = torch.zeros_like(b)
    t0 = time.perf_counter()
    rc2, rep2 = ndl.ndl_cg_solve([plan], [b], [x1], rtol=rtol, precond=1, net=net, max_iter=mi)
    torch.cuda.synchronize()
    t_learn = time.perf_counter() - t0
    plan.close()
    return {"plain": {"seconds": t_plain, "iters": rep[0].iters, "rel_res": rep[0].rel_res_fp64, "rc": rc},
            "learned": {"seconds": t_learn, "iters": rep2[0].iters, "rel_res": rep2[0].rel_res_fp64, "rc": rc2,
                        "fell_back": rep2[0].fell_back},
            "speedup": t_plain / t_learn if t_learn > 0 else None}


TRAIN_KS = (4, 8, 16, 32, 64, 96, 128, 192, 256, 384)


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seeds", type=int, default=12)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    t0 = time.perf_counter()
    data = make_pairs(args.n, range(args.seeds), ks=TRAIN_KS)
    t1 = time.perf_counter()
    net = new_net(seed=1)
    train(net, data, steps=args.steps, lr=args.lr)
    t2 = time.perf_counter()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    ndl.ndl_net_save(net, args.out)
    print(f"fields {len(data)} in {t1 - t0:.1f}s, training {t2 - t1:.1f}s -> {args.out}", flush=True)
    print(compare(net, n=args.n), flush=True)


if __name__ == "__main__":
    main()
