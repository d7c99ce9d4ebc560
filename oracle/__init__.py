"""FP64 CPU oracle for the nonlocal operators (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

The C part (``ndl_oracle.c``) holds the direct sums, the Section 3 steps and
CG; ``net_oracle.py`` holds the convolutional network reference in numpy.
Problem descriptions are plain dicts with the keys of :class:`Problem`.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libndl_oracle.so")

KERNELS = {"const": 0, "inv_r": 1, "frac": 2, "poly": 3, "cone": 4}
NORMS = {"discrete": 0, "continuous": 1, "none": 2}


class _Prob(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64), ("R", C.c_int), ("model", C.c_int),
                ("form", C.c_int), ("kernel", C.c_int), ("s", C.c_double), ("K", C.c_int),
                ("poly", C.POINTER(C.c_double)), ("norm", C.c_int), ("m2", C.c_double)]


@dataclass
class Problem:
    dim: int
    n: int
    R: int
    model: str = "diffusion"      # or "peridynamic"
    form: str = "nd"              # case (a) "nd", case (b) "div", kernel-averaged "sym"
    kernel: str = "frac"
    s: float = 0.5
    poly: Sequence[float] = field(default_factory=lambda: [1.0])
    norm: str = "discrete"
    m2: Optional[float] = None    # default 2d (diffusion) / 2d(d+2) (peridynamic)

    def second_moment(self) -> float:
        if self.m2 is not None:
            return float(self.m2)
        d = self.dim
        return 2.0 * d * (d + 2) if self.model == "peridynamic" else 2.0 * d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB)
        P = C.POINTER(_Prob)
        dp = C.POINTER(C.c_double)
        L.or_cutoff.restype = C.c_int64
        L.or_cutoff.argtypes = [C.c_double, C.c_int64]
        L.or_cutoff_pair.restype = C.c_int64
        L.or_cutoff_pair.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.or_norm.restype = C.c_double
        L.or_norm.argtypes = [P, C.c_int64, C.c_double, C.c_double]
        L.or_profile.restype = C.c_double
        L.or_profile.argtypes = [P, C.c_double]
        for f in (L.or_apply_nd, L.or_apply_div, L.or_apply_sym, L.or_fast_apply_const):
            f.restype = C.c_int
            f.argtypes = [P, dp, dp, dp, dp]
        for f in (L.or_div_diag, L.or_sym_diag):
            f.restype = C.c_int
            f.argtypes = [P, dp, dp, dp]
        L.or_decompose.restype = C.c_int64
        L.or_decompose.argtypes = [C.c_int, C.c_int64, C.POINTER(C.c_int64), C.c_int64,
                                   C.POINTER(C.c_int), C.POINTER(C.c_int64), C.c_int64]
        L.or_tree_levels.restype = C.c_int
        L.or_tree_levels.argtypes = [C.c_int64]
        L.or_tree_size.restype = C.c_int64
        L.or_tree_size.argtypes = [C.c_int, C.c_int64]
        L.or_partial_sums.restype = None
        L.or_partial_sums.argtypes = [C.c_int, C.c_int64, dp, dp]
        L.or_cg_div.restype = C.c_int
        L.or_cg_div.argtypes = [P, dp, dp, dp, dp, C.c_double, C.c_int, C.c_int,
                                C.POINTER(C.c_int), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _prob(p: Problem):
    poly = np.ascontiguousarray(np.asarray(p.poly, dtype=np.float64))
    s = _Prob(p.dim, p.n, p.R, 1 if p.model == "peridynamic" else 0,
              {"nd": 0, "div": 1, "sym": 2}[p.form], KERNELS[p.kernel], float(p.s), len(poly) - 1,
              poly.ctypes.data_as(C.POINTER(C.c_double)), NORMS[p.norm], p.second_moment())
    return s, poly


def _d(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def cutoff(delta: float, n: int) -> int:
    return int(lib().or_cutoff(float(delta), int(n)))


def cutoff_pair(di: float, dj: float, n: int) -> int:
    return int(lib().or_cutoff_pair(float(di), float(dj), int(n)))


def norm_const(p: Problem, k: int, m: float, delta: float) -> float:
    s, keep = _prob(p)
    return float(lib().or_norm(C.byref(s), int(k), float(m), float(delta)))


def profile(p: Problem, r: float) -> float:
    s, keep = _prob(p)
    return float(lib().or_profile(C.byref(s), float(r)))


def apply(p: Problem, delta, coef, u_padded) -> np.ndarray:
    """Direct sum L u.  u_padded: (ncomp, P, ..) with P = n + 2R (ncomp = dim for
    peridynamics, axis may be omitted for diffusion).  Returns (ncomp?, n, ..)."""
    s, keep = _prob(p)
    delta = _f64(delta); coef = _f64(coef); u = _f64(u_padded)
    ncomp = p.dim if p.model == "peridynamic" else 1
    out = np.zeros((ncomp,) + (p.n,) * p.dim)
    fn = {"div": lib().or_apply_div, "sym": lib().or_apply_sym, "nd": lib().or_apply_nd}[p.form]
    rc = fn(C.byref(s), _d(delta), _d(coef), _d(u), _d(out))
    if rc != 0:
        raise ValueError("oracle: collar narrower than the horizon")
    return out if p.model == "peridynamic" else out[0]


def div_diag(p: Problem, delta, coef) -> np.ndarray:
    """Diagonal of -L with a zero collar (case (b) for form "div", the
    kernel-averaged form for "sym")."""
    s, keep = _prob(p)
    delta = _f64(delta); coef = _f64(coef)
    out = np.zeros((p.n,) * p.dim)
    fn = lib().or_sym_diag if p.form == "sym" else lib().or_div_diag
    fn(C.byref(s), _d(delta), _d(coef), _d(out))
    return out


def fast_apply_const(p: Problem, delta, coef, u) -> np.ndarray:
    """The three steps of Section 3 (K = 0, zero collar); u unpadded."""
    s, keep = _prob(p)
    delta = _f64(delta); coef = _f64(coef); u = _f64(u)
    out = np.zeros((p.n,) * p.dim)
    rc = lib().or_fast_apply_const(C.byref(s), _d(delta), _d(coef), _d(u), _d(out))
    if rc != 0:
        raise ValueError("oracle: fast apply needs the constant profile, case (a), diffusion")
    return out


def decompose(dim: int, n: int, center, k: int):
    """Step 1 for one node: list of (level, (j_1..j_d)) panels of the tree over Omega."""
    c = (C.c_int64 * 3)(*(list(center) + [0] * (3 - len(center))))
    cap = 1 << 16
    lev = (C.c_int * cap)()
    idx = (C.c_int64 * (cap * dim))()
    cnt = int(lib().or_decompose(dim, n, c, int(k), lev, idx, cap))
    assert cnt <= cap
    return [(int(lev[q]), tuple(int(idx[q * dim + a]) for a in range(dim))) for q in range(cnt)]


def tree_levels(n: int) -> int:
    return int(lib().or_tree_levels(int(n)))


def partial_sums(dim: int, n: int, u) -> list:
    """Step 2: list over levels l = 0..L of arrays of shape (2^l,)*dim."""
    u = _f64(u)
    L = tree_levels(n)
    S = np.zeros(int(lib().or_tree_size(dim, n)))
    lib().or_partial_sums(dim, n, _d(u), _d(S))
    out, off = [], 0
    for l in range(L + 1):
        cnt = 1 << (dim * l)
        out.append(S[off:off + cnt].reshape((1 << l,) * dim))
        off += cnt
    return out


def cg_div(p: Problem, delta, coef, b, x0=None, rtol=1e-8, maxit=100000, jacobi=True):
    """FP64 (Jacobi-)CG for -L_div x = b, zero collar; returns (x, iters, relres, ok)."""
    s, keep = _prob(p)
    delta = _f64(delta); coef = _f64(coef); b = _f64(b)
    x = _f64(np.zeros_like(b) if x0 is None else x0).copy()
    it = C.c_int(0)
    rr = C.c_double(0.0)
    rc = lib().or_cg_div(C.byref(s), _d(delta), _d(coef), _d(b), _d(x), float(rtol), int(maxit),
                         1 if jacobi else 0, C.byref(it), C.byref(rr))
    if rc < 0:
        raise ValueError("oracle: collar narrower than the horizon")
    return x, it.value, rr.value, rc == 0
