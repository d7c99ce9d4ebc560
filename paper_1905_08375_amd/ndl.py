"""Thin ctypes binding of the C ABI in include/ndl.h (argument marshalling only).

Every computation runs in the HIP library ``libndl.so`` built next to this
file; there is no other code path.  Tensors are torch device tensors; their
data pointers and the current HIP stream are handed to the library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libndl.so")

NDL_OK, NDL_EINVAL, NDL_ENOMEM, NDL_EUNSUPPORTED, NDL_ENOTSPD, NDL_ENOCONV, NDL_EHIP, NDL_EBREAKDOWN = \
    0, -1, -2, -3, -4, -5, -6, -7
NDL_F64, NDL_F32C, NDL_F32K = 0, 1, 2
NDL_DIFFUSION, NDL_PERIDYNAMIC = 0, 1
NDL_ND, NDL_DIV, NDL_SYM = 0, 1, 2
NDL_G_CONST, NDL_G_INV_R, NDL_G_FRAC, NDL_G_POLY, NDL_G_CONE = 0, 1, 2, 3, 4
NDL_NORM_DISCRETE, NDL_NORM_CONTINUOUS, NDL_NORM_NONE = 0, 1, 2

# every symbol include/ndl.h declares
EXPORTS = [
    "ndl_plan_create", "ndl_plan_destroy", "ndl_plan_get_info", "ndl_apply", "ndl_apply_fast",
    "ndl_fast_decomposition", "ndl_decompose_node", "ndl_cg_solve", "ndl_net_create", "ndl_net_destroy", "ndl_net_set_linear",
    "ndl_net_save", "ndl_net_load", "ndl_net_num_params", "ndl_net_train_step", "ndl_precond_apply",
    "ndl_autotune", "ndl_last_error", "ndl_version", "ndl_plan_set_variant", "ndl_plan_num_variants",
    "ndl_net_conv_test", "ndl_net_train_step_energy", "ndl_net_layer_tensor", "ndl_apply_fast_noalloc",
    "ndl_autotune_apply", "ndl_div_batch_apply", "ndl_plan_set_fast_method",
]


class ndl_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int64), ("collar", C.c_int32), ("model", C.c_int32),
                ("form", C.c_int32), ("kernel", C.c_int32), ("s", C.c_double), ("K", C.c_int32),
                ("poly", C.POINTER(C.c_double)), ("norm", C.c_int32), ("m2_target", C.c_double),
                ("prec", C.c_int32), ("delta", C.c_void_p), ("coef", C.c_void_p)]


class ndl_plan_info(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("k_max", C.c_int64), ("k_min", C.c_int64), ("ncomp", C.c_int32),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32), ("variant", C.c_int32),
                ("fast_levels", C.c_int32), ("pairs_per_point", C.c_double), ("pair_order", C.c_int32),
                ("fast_method", C.c_int32)]


class ndl_cg_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precond", C.c_int32), ("net", C.c_void_p),
                ("graph_iters", C.c_int32), ("inner_rtol", C.c_double), ("use_fast", C.c_int32)]


class ndl_cg_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("converged", C.c_int32), ("fell_back", C.c_int32),
                ("rel_res_fp64", C.c_double), ("seconds", C.c_double)]


class NdlError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


_lib = None


def lib():
    """Load libndl.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: run __graft_entry__.build() (no fallback path exists)")
        # torch first: the library then binds to the HIP runtime torch already
        # loaded, so that one process holds one runtime (two copies of it do
        # not share devices)
        import torch  # noqa: F401
        L = C.CDLL(LIBPATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "ndl_plan_create": [C.POINTER(ndl_problem), C.c_int, C.POINTER(vp), vp],
            "ndl_plan_destroy": [vp],
            "ndl_plan_get_info": [vp, C.POINTER(ndl_plan_info)],
            "ndl_apply": [vp, vp, vp, C.c_int, vp],
            "ndl_apply_fast": [vp, vp, vp, C.c_int, vp],
            "ndl_apply_fast_noalloc": [vp, vp, vp, C.c_int, vp],
            "ndl_fast_decomposition": [vp, C.POINTER(i64), C.POINTER(i32), i32, C.POINTER(i32)],
            "ndl_decompose_node": [i32, i64, C.POINTER(i64), i64, C.POINTER(i32), i32, C.POINTER(i32)],
            "ndl_cg_solve": [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(ndl_cg_opts),
                             C.POINTER(ndl_cg_report), vp],
            "ndl_net_create": [C.c_int, C.POINTER(C.c_int), C.c_uint64, C.POINTER(vp)],
            "ndl_net_destroy": [vp],
            "ndl_net_set_linear": [vp, C.c_int32],
            "ndl_net_save": [vp, C.c_char_p],
            "ndl_net_load": [vp, C.c_char_p],
            "ndl_net_num_params": [vp, C.POINTER(i64)],
            "ndl_net_train_step": [vp, C.c_int, C.c_int, vp, vp, vp, C.c_float, C.POINTER(C.c_float), vp],
            "ndl_precond_apply": [vp, vp, vp, vp, vp],
            "ndl_autotune": [vp, vp],
            "ndl_autotune_apply": [vp, vp, C.c_int, vp],
            "ndl_div_batch_apply": [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.c_int,
                                    C.POINTER(C.c_int), C.POINTER(C.c_int), vp],
            "ndl_plan_set_variant": [vp, C.c_int],
            "ndl_plan_set_fast_method": [vp, C.c_int],
            "ndl_plan_num_variants": [vp, C.POINTER(C.c_int)],
            "ndl_net_train_step_energy": [vp, vp, C.c_int, vp, vp, C.c_float, C.POINTER(C.c_float), vp],
            "ndl_net_conv_test": [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "ndl_net_layer_tensor": [vp, C.c_int, C.c_int, C.POINTER(C.c_float), i64],
        }
        for name, args in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = C.c_int
        L.ndl_last_error.restype = C.c_char_p
        L.ndl_last_error.argtypes = []
        L.ndl_version.restype = C.c_char_p
        L.ndl_version.argtypes = []
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != NDL_OK:
        raise NdlError(rc, where, lib().ndl_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


class Plan:
    """Owns an ndl_plan handle and keeps its delta/coef tensors alive."""

    def __init__(self, handle, prob, keep):
        self.handle = handle
        self.prob = prob
        self._keep = keep

    def info(self) -> ndl_plan_info:
        inf = ndl_plan_info()
        _check(lib().ndl_plan_get_info(self.handle, C.byref(inf)), "ndl_plan_get_info")
        return inf

    def close(self):
        if self.handle:
            lib().ndl_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_problem(dim, n, collar, delta, coef, *, model=NDL_DIFFUSION, form=NDL_ND, kernel=NDL_G_FRAC,
                 s=0.5, poly: Sequence[float] = (1.0,), norm=NDL_NORM_DISCRETE, m2_target=0.0, prec=NDL_F32C):
    pa = (C.c_double * len(poly))(*poly)
    p = ndl_problem(dim, n, collar, model, form, kernel, s, len(poly) - 1, pa, norm, m2_target, prec,
                    _ptr(delta), _ptr(coef))
    p._poly_keep = pa
    return p


def ndl_plan_create(prob: ndl_problem, want_fast: int = 0, stream=None, keep=()) -> Plan:
    """want_fast: 0 direct only, 1 (or True) with the hierarchical path and its
    pyramid workspace, 2 hierarchical path without it (ndl_apply_fast_noalloc)."""
    h = C.c_void_p()
    _check(lib().ndl_plan_create(C.byref(prob), int(want_fast), C.byref(h), _stream(stream)),
           "ndl_plan_create")
    return Plan(h, prob, keep)


def ndl_plan_destroy(plan: Plan):
    plan.close()


def ndl_apply(plan: Plan, u, Lu, batch: int = 1, stream=None):
    _check(lib().ndl_apply(plan.handle, _ptr(u), _ptr(Lu), int(batch), _stream(stream)), "ndl_apply")


def ndl_apply_fast(plan: Plan, u, Lu, batch: int = 1, stream=None):
    _check(lib().ndl_apply_fast(plan.handle, _ptr(u), _ptr(Lu), int(batch), _stream(stream)), "ndl_apply_fast")


def ndl_apply_fast_noalloc(plan: Plan, u, Lu, batch: int = 1, stream=None):
    _check(lib().ndl_apply_fast_noalloc(plan.handle, _ptr(u), _ptr(Lu), int(batch), _stream(stream)),
           "ndl_apply_fast_noalloc")


def _records(buf, cnt, dim):
    return [(int(buf[q * (dim + 1)]), tuple(int(buf[q * (dim + 1) + 1 + a]) for a in range(dim)))
            for q in range(cnt)]


def ndl_fast_decomposition(plan: Plan, node: Sequence[int], cap: int = 1 << 16):
    dim = len(node)
    nd = (C.c_int64 * dim)(*node)
    buf = (C.c_int32 * (cap * (dim + 1)))()
    cnt = C.c_int32()
    _check(lib().ndl_fast_decomposition(plan.handle, nd, buf, cap, C.byref(cnt)), "ndl_fast_decomposition")
    return _records(buf, min(cnt.value, cap), dim)


def ndl_decompose_node(dim: int, n: int, node: Sequence[int], k: int, cap: int = 1 << 16):
    nd = (C.c_int64 * dim)(*node)
    buf = (C.c_int32 * (cap * (dim + 1)))()
    cnt = C.c_int32()
    _check(lib().ndl_decompose_node(dim, n, nd, k, buf, cap, C.byref(cnt)), "ndl_decompose_node")
    return _records(buf, min(cnt.value, cap), dim)


def ndl_plan_set_variant(plan: Plan, variant: int):
    _check(lib().ndl_plan_set_variant(plan.handle, int(variant)), "ndl_plan_set_variant")


def ndl_plan_set_fast_method(plan: Plan, method: int):
    _check(lib().ndl_plan_set_fast_method(plan.handle, int(method)), "ndl_plan_set_fast_method")


def ndl_plan_num_variants(plan: Plan) -> int:
    c = C.c_int()
    _check(lib().ndl_plan_num_variants(plan.handle, C.byref(c)), "ndl_plan_num_variants")
    return c.value


def ndl_autotune(plan: Plan, stream=None):
    _check(lib().ndl_autotune(plan.handle, _stream(stream)), "ndl_autotune")
    return plan.info()


def ndl_autotune_apply(plan: Plan, u, batch: int = 1, stream=None):
    _check(lib().ndl_autotune_apply(plan.handle, _ptr(u), int(batch), _stream(stream)), "ndl_autotune_apply")
    return plan.info()


def ndl_div_batch_apply(plans: Sequence[Plan], x_list, y_list, variant: int = -1, stream=None):
    """y_i = -L x_i for case (b) plans in one batched launch; returns (variant used, number of variants)."""
    n = len(plans)
    ph = (C.c_void_p * n)(*[p.handle.value if isinstance(p.handle, C.c_void_p) else p.handle for p in plans])
    xp = (C.c_void_p * n)(*[_ptr(x) for x in x_list])
    yp = (C.c_void_p * n)(*[_ptr(y) for y in y_list])
    used, nv = C.c_int(), C.c_int()
    _check(lib().ndl_div_batch_apply(ph, n, xp, yp, int(variant), C.byref(used), C.byref(nv), _stream(stream)),
           "ndl_div_batch_apply")
    return used.value, nv.value


def ndl_cg_solve(plans: Sequence[Plan], b_list, x_list, rtol=1e-8, max_iter=200000, precond=0, net=None,
                 graph_iters=0, inner_rtol=0.0, use_fast=False, stream=None):
    n = len(plans)
    ph = (C.c_void_p * n)(*[p.handle.value if isinstance(p.handle, C.c_void_p) else p.handle for p in plans])
    bp = (C.c_void_p * n)(*[_ptr(b) for b in b_list])
    xp = (C.c_void_p * n)(*[_ptr(x) for x in x_list])
    opts = ndl_cg_opts(rtol, max_iter, precond, net.handle if net is not None else None, graph_iters, inner_rtol,
                       int(bool(use_fast)))
    reps = (ndl_cg_report * n)()
    rc = lib().ndl_cg_solve(ph, n, bp, xp, C.byref(opts), reps, _stream(stream))
    if rc not in (NDL_OK, NDL_ENOCONV):
        _check(rc, "ndl_cg_solve")
    return rc, [reps[i] for i in range(n)]


def ndl_last_error() -> str:
    return lib().ndl_last_error().decode()


def ndl_version() -> str:
    return lib().ndl_version().decode()


# ---------------------------------------------------------------- learned preconditioner
class Net:
    """Owns an ndl_net handle."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().ndl_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ndl_net_create(levels: int = 4, channels=(16, 16, 32, 32), seed: int = 0) -> Net:
    h = C.c_void_p()
    ch = (C.c_int * len(channels))(*channels)
    _check(lib().ndl_net_create(int(levels), ch, C.c_uint64(seed), C.byref(h)), "ndl_net_create")
    return Net(h)


def ndl_net_set_linear(net: Net, linear: bool = True):
    _check(lib().ndl_net_set_linear(net.handle, int(bool(linear))), "ndl_net_set_linear")


def ndl_net_destroy(net: Net):
    net.close()


def ndl_net_num_params(net: Net) -> int:
    c = C.c_int64()
    _check(lib().ndl_net_num_params(net.handle, C.byref(c)), "ndl_net_num_params")
    return c.value


def ndl_net_save(net: Net, path: str):
    _check(lib().ndl_net_save(net.handle, path.encode()), "ndl_net_save")


def ndl_net_load(net: Net, path: str):
    _check(lib().ndl_net_load(net.handle, path.encode()), "ndl_net_load")


def ndl_net_train_step(net: Net, r, feat, e, lr: float, stream=None) -> float:
    """r, e: [B][s,s,s] fp32; feat: [B][2][s,s,s] fp32 (device)."""
    B, s = r.shape[0], r.shape[-1]
    loss = C.c_float()
    _check(lib().ndl_net_train_step(net.handle, int(B), int(s), _ptr(r), _ptr(feat), _ptr(e), C.c_float(lr),
                                    C.byref(loss), _stream(stream)), "ndl_net_train_step")
    return loss.value


def ndl_precond_apply(net: Net, plan: Plan, r, z, stream=None):
    _check(lib().ndl_precond_apply(net.handle, plan.handle, _ptr(r), _ptr(z), _stream(stream)), "ndl_precond_apply")


def ndl_net_conv_test(cin, cout, S, x_bits, w, bias, y=None, dy=None, dx=None, gw=None, gb=None, stream=None):
    _check(lib().ndl_net_conv_test(int(cin), int(cout), int(S), _ptr(x_bits), _ptr(w), _ptr(bias), _ptr(y), _ptr(dy),
                                   _ptr(dx), _ptr(gw), _ptr(gb), _stream(stream)), "ndl_net_conv_test")


def ndl_net_train_step_energy(net: Net, plan: Plan, r, e, lr: float, stream=None) -> float:
    """r, e: [B][n,n,n] fp32 device tensors on the plan's grid (A e = r)."""
    loss = C.c_float()
    _check(lib().ndl_net_train_step_energy(net.handle, plan.handle, int(r.shape[0]), _ptr(r), _ptr(e), C.c_float(lr),
                                           C.byref(loss), _stream(stream)), "ndl_net_train_step_energy")
    return loss.value


# which tensor ndl_net_layer_tensor reads
NET_W, NET_B, NET_GW, NET_GB, NET_MW, NET_VW, NET_MB, NET_VB = range(8)
_NET_COUT = (16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16, 16)
_NET_CIN = (8, 16, 16, 16, 16, 32, 32, 32, 32, 32, 16, 16, 16)


def ndl_net_layer_tensor(net: Net, layer: int, which: int):
    """A layer's FP32 tensor as a numpy array: [cout][KP] for weights and
    their gradient and moments, [cout] for biases and theirs."""
    import numpy as np
    cout = _NET_COUT[layer]
    kp = ((27 * _NET_CIN[layer] + 31) // 32) * 32
    shape = (cout,) if which in (NET_B, NET_GB, NET_MB, NET_VB) else (cout, kp)
    out = np.zeros(shape, dtype=np.float32)
    _check(lib().ndl_net_layer_tensor(net.handle, int(layer), int(which),
                                      out.ctypes.data_as(C.POINTER(C.c_float)), int(out.size)),
           "ndl_net_layer_tensor")
    return out
