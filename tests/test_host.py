"""CPU-only checks of the library: it loads, exports the ABI, and its Step 1
routine (evaluated on the host) reproduces the oracle's Algorithm recur."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1905_08375_amd import ndl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "ndl.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ndl_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = ndl.lib()
    syms = header_symbols()
    assert len(syms) >= 15
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert sorted(syms) == sorted(ndl.EXPORTS)
    assert "gfx950" in ndl.ndl_version()


def to_oracle(recs, n):
    L = O.tree_levels(n)
    return sorted((L - s, j) for s, j in recs)


@pytest.mark.parametrize("dim,n,ks", [
    (1, 64, [0, 3, 30, 200, 5000]),
    (1, 100, [7, 64, 2000]),
    (2, 32, [0, 1, 8, 35, 150, 2000]),
    (2, 24, [35, 150]),
    (2, 128, [1023, 4095]),
    (3, 16, [3, 12, 35, 200]),
    (3, 12, [20]),
])
def test_step1_matches_algorithm_recur(dim, n, ks):
    g = np.random.default_rng(dim * 1000 + n)
    for k in ks:
        centers = [tuple([0] * dim), tuple([n - 1] * dim)] + [tuple(g.integers(0, n, dim)) for _ in range(6)]
        for c in centers:
            got = to_oracle(ndl.ndl_decompose_node(dim, n, c, k), n)
            want = sorted(O.decompose(dim, n, c, k))
            assert got == want, (dim, n, k, c)


def test_step1_rejects_bad_node():
    with pytest.raises(ndl.NdlError):
        ndl.ndl_decompose_node(2, 16, (16, 0), 8)
