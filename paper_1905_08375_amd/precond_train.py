"""Training and evaluation of the learned preconditioner (3D case (b) workload).

Training pairs come from plain Jacobi-CG runs of the library on seeded fields:
for each training field the solver is run to a tight tolerance (x*) and, from
the same start, for k = k_1 < k_2 < ... iterations (x_k); the pair is the
residual r_k = b + L x_k and the correction e_k = x* - x_k on the whole
field.  The network is trained on full fields with the energy norm that CG
minimises: for the two-level preconditioner z = D^-1 r + M(r) the loss is
||e - z||_A^2 / ||e||_A^2 (A = -L), evaluated with the library's operator.
Every arithmetic step runs in libndl (the operator, the solves, the
network's forward/backward and Adam); torch only holds the tensors.
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


def cg_iterate(plan, b, iters, rtol=1e-10):
    import torch
    x = torch.zeros_like(b)
    ndl.ndl_cg_solve([plan], [b], [x], rtol=rtol, max_iter=iters)
    return x


def make_pairs(n=256, seeds=range(8), ks=(8, 16, 32, 64, 128, 256), log=print):
    """Per training field: its plan and the CG pairs (r_k, e_k) as FP32 fields."""
    import torch
    out = []
    for sd in seeds:
        t0 = time.perf_counter()
        plan, b, feat, _ = problem_3d(n, sd)
        xs = cg_iterate(plan, b, 100000, rtol=1e-9)
        pairs = []
        for k in ks:
            xk = cg_iterate(plan, b, k)
            ek = (xs - xk).float()
            rk = (b - neg_L(plan, xk, n)).float()
            pairs.append((rk, ek))
        out.append((plan, pairs))
        log(f"pairs: seed {sd} done in {time.perf_counter() - t0:.1f}s")
    return out


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


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    t0 = time.perf_counter()
    data = make_pairs(args.n, range(args.seeds))
    t1 = time.perf_counter()
    net = ndl.ndl_net_create(seed=1)
    train(net, data, steps=args.steps)
    t2 = time.perf_counter()
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    ndl.ndl_net_save(net, args.out)
    print(f"fields {len(data)} in {t1 - t0:.1f}s, training {t2 - t1:.1f}s -> {args.out}", flush=True)
    print(compare(net, n=args.n), flush=True)


if __name__ == "__main__":
    main()
