"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact lattice
identities, closed forms, a library convolution, brute-force set properties,
matrix symmetry/definiteness, or a second route through the Section 3 steps.
"""
import math
import os

import numpy as np
import pytest
from scipy import signal

import oracle as O
from paper_1905_08375_amd import fields as F

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_fields(n, dim, mlo, mhi, seed):
    g = np.random.default_rng(seed)
    m = g.uniform(mlo, mhi, (n,) * dim)
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    return m / n, c


KERNELS = [("const", {}), ("inv_r", {}), ("frac", {"s": 0.5}), ("frac", {"s": 0.25}),
           ("poly", {"poly": [2.1875, -2.1875, 1.3125, -0.3125]}), ("cone", {})]


# --------------------------------------------------------------- P1
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("form", ["nd", "div"])
def test_constant_in_kernel(dim, form):
    """L of a constant (collar holding the same constant) is exactly 0."""
    n = {1: 40, 2: 14, 3: 7}[dim]
    R = 4
    P = O.Problem(dim=dim, n=n, R=R, form=form, kernel="frac")
    delta, c = rand_fields(n, dim, 1.2, 4.0, 1)
    u = np.full((n + 2 * R,) * dim, -2.375)
    assert np.all(O.apply(P, delta, c, u) == 0.0)


@pytest.mark.parametrize("dim,kname", [(2, "inv_r"), (2, "cone"), (3, "inv_r"), (3, "cone")])
def test_pd_rigid_translation_exact_zero(dim, kname):
    n, R = {2: 14, 3: 7}[dim], 5
    P = O.Problem(dim=dim, n=n, R=R, model="peridynamic", kernel=kname)
    delta, c = rand_fields(n, dim, 2.0, 5.0, 2)
    u = np.empty((dim,) + (n + 2 * R,) * dim)
    for a, v in enumerate([0.3, -1.7, 0.9][:dim]):
        u[a] = v
    assert np.all(O.apply(P, delta, c, u) == 0.0)


@pytest.mark.parametrize("dim,kname", [(2, "inv_r"), (2, "cone"), (3, "inv_r"), (3, "frac")])
def test_pd_infinitesimal_rotation_zero(dim, kname):
    """u = W (x - x0) with W antisymmetric (an infinitesimal rotation): every
    bond stretch e.(W z) vanishes (Section 1 linear force), so L u = 0 up to
    rounding; in 3D about an axis that is no lattice axis."""
    n, R = {2: 16, 3: 8}[dim], 6
    P = O.Problem(dim=dim, n=n, R=R, model="peridynamic", kernel=kname, s=0.5)
    delta, c = rand_fields(n, dim, 2.0, 6.0, 3)
    X = F.padded_coords(n, dim, R)
    x0 = [0.31, 0.77, 0.45][:dim]
    if dim == 2:
        W = np.array([[0.0, -0.37], [0.37, 0.0]])
    else:
        W = np.array([[0.0, -0.37, 0.21], [0.37, 0.0, -0.55], [-0.21, 0.55, 0.0]])
    u = np.stack([sum(W[a, b] * (X[b] - x0[b]) for b in range(dim)) for a in range(dim)])
    Lu = O.apply(P, delta, c, u)
    scale = np.abs(c).max() * 2 * dim * (dim + 2) * n * n * 0.6 / n  # |omega| h^d |du| order
    assert np.abs(Lu).max() < 1e-12 * scale


# --------------------------------------------------------------- P2
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("kname,kw", KERNELS)
def test_quadratic_reproduces_laplacian(dim, kname, kw):
    """Discrete normalisation: L |x|^2 = 2d c exactly and L x_1^2 = 2 c (case (a) limit
    C(x) Delta u, Section 2); the collar carries the quadratic."""
    n = {1: 48, 2: 14, 3: 7}[dim]
    R = 5
    P = O.Problem(dim=dim, n=n, R=R, kernel=kname, **kw)
    delta, c = rand_fields(n, dim, 1.1, 5.0, 4 + dim)
    X = F.padded_coords(n, dim, R)
    r2 = sum(x * x for x in X)
    assert np.allclose(O.apply(P, delta, c, r2), 2 * dim * c, rtol=1e-12, atol=0)
    assert np.allclose(O.apply(P, delta, c, X[0] ** 2), 2 * c, rtol=1e-12, atol=0)
    # a linear field is annihilated (odd moments cancel on the symmetric ball)
    lin = 0.7 * X[0] - 0.2 * X[-1] + 3.0
    assert np.abs(O.apply(P, delta, c, lin)).max() < 1e-9 * n


@pytest.mark.parametrize("dim,kname", [(2, "inv_r"), (2, "cone"), (3, "inv_r"), (3, "cone")])
def test_pd_quadratic_identity(dim, kname):
    """Peridynamics with M = 2d(d+2): L (|x|^2, 0, ..) = (M/d c, 0, ..) exactly
    on the lattice (the ball is symmetric under axis permutations, so the
    z_1^2-weighted sum is 1/d of the normalised second moment)."""
    n, R = {2: 16, 3: 8}[dim], 7
    P = O.Problem(dim=dim, n=n, R=R, model="peridynamic", kernel=kname)
    delta, c = rand_fields(n, dim, 2.0, 7.0, 9)
    X = F.padded_coords(n, dim, R)
    u = np.stack([sum(x * x for x in X)] + [np.zeros_like(X[0])] * (dim - 1))
    Lu = O.apply(P, delta, c, u)
    M = 2 * dim * (dim + 2)
    assert np.allclose(Lu[0], M / dim * c, rtol=1e-12)
    for a in range(1, dim):
        assert np.abs(Lu[a]).max() < 1e-11 * M


def test_pd_local_limit_navier():
    """L (x_1^2, 0) tends to c (Delta u + 2 grad div u) = (6c, 0) as the horizon grows."""
    n, R = 6, 40
    P = O.Problem(dim=2, n=n, R=R, model="peridynamic", kernel="inv_r")
    delta = np.full((n, n), 39.5 / n)
    c = np.ones((n, n))
    X1, X2 = F.padded_coords(n, 2, R)
    Lu = O.apply(P, delta, c, np.stack([X1 ** 2, 0 * X1]))
    assert abs(Lu[0].mean() - 6.0) < 0.02


# --------------------------------------------------------------- P3
def assemble(P, delta, c):
    n, d, R = P.n, P.dim, P.R
    N = n ** d
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros((n,) * d)
        e.flat[j] = 1.0
        A[:, j] = O.apply(P, delta, c, F.pad(e, R)).ravel()
    return A


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 5)])
def test_div_symmetric_negative_definite(dim, n):
    R = 4
    P = O.Problem(dim=dim, n=n, R=R, form="div", kernel="frac")
    delta, c = rand_fields(n, dim, 2.0, 4.0, 11)
    A = assemble(P, delta, c)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    np.linalg.cholesky(-A)  # -L_div is SPD under a zero volume constraint
    # diagonal helper equals -A_ii
    assert np.allclose(O.div_diag(P, delta, c).ravel(), -np.diag(A), rtol=1e-13)


def test_nd_not_symmetric():
    """Case (a) with variable delta, C is non-symmetric (the paper's heterogeneous tests)."""
    n, R = 12, 4
    P = O.Problem(dim=2, n=n, R=R, kernel="frac")
    delta, c = rand_fields(n, 2, 2.0, 4.0, 12)
    A = assemble(P, delta, c)
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


# --------------------------------------------------------------- P4
@pytest.mark.parametrize("kname,kw", KERNELS)
def test_constant_coefficients_are_a_convolution(kname, kw):
    """Constant delta and C: L u = w * u - (sum w) u, a zero-padded linear convolution
    computed with scipy's FFT convolution (the translation-invariant case)."""
    n, R, m = 40, 5, 4.3
    P = O.Problem(dim=2, n=n, R=R, kernel=kname, **kw)
    delta = np.full((n, n), m / n)
    c = np.full((n, n), 1.7)
    g = np.random.default_rng(13)
    u = g.standard_normal((n, n))
    J = 4
    z = np.arange(-J, J + 1)
    Z1, Z2 = np.meshgrid(z, z, indexing="ij")
    q = Z1 ** 2 + Z2 ** 2
    k = math.ceil((m) ** 2) - 1
    inside = (q > 0) & (q <= k)
    r = np.sqrt(np.where(inside, q, 1)) / m
    if kname == "const":
        prof = np.ones_like(r)
    elif kname == "inv_r":
        prof = 1 / r
    elif kname == "poly":
        # even polynomial sum_j a_j r^(2j) (the p^{2K} of Section 3), Horner in r^2
        prof = np.zeros_like(r)
        for a in reversed(kw["poly"]):
            prof = prof * r * r + a
    elif kname == "cone":
        prof = (1 - r) / r  # the conical micromodulus of eq. "kernelgamma"
    else:
        prof = r ** (-(2 + 2 * kw["s"]))
    prof = np.where(inside, prof, 0.0)
    h = 1.0 / n
    A = 4.0 / np.sum(prof * q * h * h * h * h)
    w = 1.7 * A * prof * h * h
    conv = signal.fftconvolve(u, w[::-1, ::-1], mode="same")  # correlation = convolution w/ flip
    ref = conv - w.sum() * u
    got = O.apply(P, delta, c, F.pad(u, R))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# --------------------------------------------------------------- case (b) normalisation
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("kname,kw", KERNELS[:4])
def test_div_with_constant_fields_is_case_a(dim, kname, kw):
    """Case (b) with constant delta and C: delta_ij = delta and C_ij = C, so the
    symmetric operator is case (a) itself and reproduces the local limit, L |x|^2 =
    2d c exactly (Section 2, cases (a) and (b)).  The case (b) side takes its
    normalisation per cutoff from moment sums memoised by k, the case (a) side
    enumerates the ball per node: two independent routes to A(k, m)."""
    n = {1: 40, 2: 13, 3: 6}[dim]
    R = 5
    m = {1: 4.7, 2: 3.3, 3: 2.6}[dim]
    delta = np.full((n,) * dim, m / n)
    c = np.full((n,) * dim, 1.37)
    g = np.random.default_rng(40 + dim)
    u = g.standard_normal((n + 2 * R,) * dim)
    Pa = O.Problem(dim=dim, n=n, R=R, form="nd", kernel=kname, **kw)
    Pb = O.Problem(dim=dim, n=n, R=R, form="div", kernel=kname, **kw)
    La, Lb = O.apply(Pa, delta, c, u), O.apply(Pb, delta, c, u)
    assert np.abs(La - Lb).max() <= 1e-13 * np.abs(La).max()
    X = F.padded_coords(n, dim, R)
    r2 = sum(x * x for x in X)
    assert np.allclose(O.apply(Pb, delta, c, r2), 2 * dim * 1.37, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim,n", [(1, 30), (2, 8), (3, 5)])
@pytest.mark.parametrize("kname,kw", [("frac", {"s": 0.5}), ("inv_r", {}), ("const", {})])
def test_div_pair_weight_is_case_a_at_the_mean_horizon(dim, n, kname, kw):
    """Every entry of the assembled case (b) matrix, A_ij for j != i, is the case
    (a) entry of the constant-field problem with delta = (delta_i + delta_j)/2 and
    C = (c_i + c_j)/2 (Section 2, case (b) with the symmetric C and delta): the
    pair weight is the full normalised kernel evaluated at the pair's mean
    horizon, including its cutoff k_ij."""
    R = 4
    g = np.random.default_rng(50 + dim)
    delta = g.uniform(1.3, 4.0, (n,) * dim) / n
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    Pb = O.Problem(dim=dim, n=n, R=R, form="div", kernel=kname, **kw)
    A = assemble(Pb, delta, c)
    N = n ** dim
    Pa = O.Problem(dim=dim, n=n, R=R, form="nd", kernel=kname, **kw)
    for i in g.choice(N, size=4, replace=False):
        row = A[i]
        js = [j for j in range(N) if j != i]
        for j in g.choice(js, size=min(8, len(js)), replace=False):
            dm = 0.5 * (delta.flat[i] + delta.flat[j])
            cm = 0.5 * (c.flat[i] + c.flat[j])
            e = np.zeros((n,) * dim)
            e.flat[j] = 1.0
            ref = O.apply(Pa, np.full((n,) * dim, dm), np.full((n,) * dim, cm), F.pad(e, R)).flat[i]
            assert abs(row[j] - ref) <= 1e-13 * max(abs(ref), abs(A[i, i])), (i, j, row[j], ref)


# --------------------------------------------------------------- P5
def test_1d_sines_closed_form():
    """1D, constant kernel 3/delta^3, delta = 0.01, n = 4096 (J = 40 neighbours per side):
    at interior nodes L sin(pi f x) = A h sin(pi f x)[D_J(theta) - (2J+1)], theta = pi f h,
    with the Dirichlet kernel D_J(theta) = sin((J+1/2) theta)/sin(theta/2)."""
    d = F.diffusion_1d()
    n, R = 4096, 41
    P = O.Problem(dim=1, n=n, R=R, kernel="const", norm="continuous")
    assert O.cutoff(0.01, n) == 1677 and math.isqrt(1677) == 40
    Lu = O.apply(P, d["delta"], d["coef"], F.pad(d["u"], R))
    x = F.nodes(n)
    h, A, J = 1.0 / n, 3.0 / 0.01 ** 3, 40
    ref = np.zeros(n)
    for a, f in zip(d["amps"], d["freqs"]):
        th = np.pi * f * h
        ref += a * A * h * np.sin(np.pi * f * x) * (np.sin((J + 0.5) * th) / np.sin(th / 2) - (2 * J + 1))
    sl = slice(J, n - J)
    assert np.abs(Lu[sl] - ref[sl]).max() <= 1e-12 * np.abs(ref[sl]).max()


def test_continuous_constant_matches_3_over_delta_cubed():
    P = O.Problem(dim=1, n=4096, R=41, kernel="const", norm="continuous")
    assert O.norm_const(P, 1677, 40.96, 0.01) == pytest.approx(3.0 / 0.01 ** 3, rel=1e-14)


# --------------------------------------------------------------- cutoff
def test_cutoff_is_strict():
    n = 64
    for m in [2.0, 3.0, 4.0, 2.5, 2.25, 5.5, 6.0]:
        k = O.cutoff(m / n, n)
        # |z|^2 < m^2 on the integer lattice
        assert all((q <= k) == (q < m * m - 1e-9) for q in range(0, 60)), m
    assert O.cutoff_pair(2.0 / n, 4.0 / n, n) == 8


# --------------------------------------------------------------- P8
def ball_nodes(dim, n, c, k):
    R = math.isqrt(k)
    pts = set()
    rng_ = [range(-R, R + 1)] * dim
    for z in np.ndindex(*([2 * R + 1] * dim)):
        zz = [v - R for v in z]
        y = [c[a] + zz[a] for a in range(dim)]
        if sum(v * v for v in zz) <= k and all(0 <= v < n for v in y):
            pts.add(tuple(y))
    return pts


def panel_nodes(dim, n, lev, j):
    L = O.tree_levels(n)
    side = 1 << (L - lev)
    axes = [range(j[a] * side, (j[a] + 1) * side) for a in range(dim)]
    return [tuple(p) for p in np.array(np.meshgrid(*axes, indexing="ij")).reshape(dim, -1).T]


@pytest.mark.parametrize("dim,n,k,centers", [
    (1, 64, 30, [(0,), (5,), (31,), (63,)]),
    (2, 32, 35, [(0, 0), (3, 17), (16, 16), (31, 2), (9, 30)]),
    (2, 24, 150, [(0, 0), (11, 12), (23, 5)]),      # n not a power of two
    (3, 16, 12, [(0, 0, 0), (7, 8, 9), (15, 3, 8)]),
])
def test_decomposition_is_exact_partition(dim, n, k, centers):
    """Step 1 (Algorithms recur + doesCubeIntersectBall on node boxes): the panels
    cover the lattice ball cut by Omega exactly once, and each panel is maximal
    (its parent is not fully inside)."""
    L = O.tree_levels(n)
    for c in centers:
        dec = O.decompose(dim, n, c, k)
        want = ball_nodes(dim, n, c, k)
        got = []
        for lev, j in dec:
            got.extend(panel_nodes(dim, n, lev, j))
        assert len(got) == len(set(got)), "overlapping panels"
        assert set(got) == want
        keys = {(lev, j) for lev, j in dec}
        for lev, j in dec:
            if lev == 0:
                continue
            par = tuple(v // 2 for v in j)
            sibs = [(lev, tuple(2 * par[a] + (mm >> a & 1) for a in range(dim)))
                    for mm in range(1 << dim)]
            assert not all(s in keys for s in sibs), "parent should have been taken whole"


def test_decomposition_size_grows_like_m():
    """About 7m panels per interior node in 2D (boundary panels dominate, Step 1 count)."""
    n = 256
    sizes = []
    for m in [8, 16, 32]:
        k = math.ceil(m * m) - 1
        cnt = [len(O.decompose(2, n, (128 + a, 128 + b), k)) for a in range(4) for b in range(4)]
        sizes.append(np.mean(cnt))
    r1, r2 = sizes[1] / sizes[0], sizes[2] / sizes[1]
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, sizes


# --------------------------------------------------------------- Section 3 route
@pytest.mark.parametrize("dim,n", [(1, 100), (2, 24), (2, 32), (3, 10)])
def test_three_steps_equal_direct_sum(dim, n):
    """Steps 1-3 with eq. nonlocalP reproduce the direct sum with a zero collar."""
    R = 7
    P = O.Problem(dim=dim, n=n, R=R, kernel="const", norm="none")
    g = np.random.default_rng(21 + dim)
    delta = g.uniform(1.0, 6.5, (n,) * dim) / n
    c = np.exp(g.normal(0, 0.3, (n,) * dim))
    u = g.standard_normal((n,) * dim)
    ref = O.apply(P, delta, c, F.pad(u, R))
    got = O.fast_apply_const(P, delta, c, u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_partial_sums_levels():
    g = np.random.default_rng(5)
    u = g.standard_normal((12, 12))
    S = O.partial_sums(2, 12, u)
    assert S[0].shape == (1, 1) and abs(S[0][0, 0] - u.sum()) < 1e-12
    up = np.zeros((16, 16)); up[:12, :12] = u
    assert np.allclose(S[2], up.reshape(4, 4, 4, 4).sum(axis=(1, 3)))


# --------------------------------------------------------------- P9
def test_polynomial_split_matches_inverse_r():
    """p^{2K} matches 1/s and its first K derivatives at s = 1 (Section 3)."""
    rows = {}
    for line in open(os.path.join(GOLD, "p2k_inv_r.txt")):
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            rows[parts[0]] = [float(v) for v in parts[1:]]
    for K in range(4):
        a = rows[str(K)]
        coeffs = np.zeros(2 * K + 1)
        coeffs[0::2] = a
        poly = np.polynomial.Polynomial(coeffs)
        for j in range(K + 1):
            want = (-1) ** j * math.factorial(j)  # d^j/ds^j s^-1 at 1
            assert poly.deriv(j)(1.0) == pytest.approx(want, abs=1e-12), (K, j)
    printed = rows["printed3"]
    c = np.zeros(7); c[0::2] = printed
    assert np.polynomial.Polynomial(c).deriv(3)(1.0) == pytest.approx(-3.0)


# --------------------------------------------------------------- P10
def disk_square_area(cx, cy, r):
    from scipy import integrate

    def chord(x):
        hw = math.sqrt(max(r * r - (x - cx) ** 2, 0.0))
        return max(0.0, min(1.0, cy + hw) - max(0.0, cy - hw))
    a, b = max(0.0, cx - r), min(1.0, cx + r)
    pts = [p for p in (cx,) if a < p < b]
    return integrate.quad(chord, a, b, points=pts or None, limit=200, epsabs=1e-13)[0]


def test_example1_boundary_convergence():
    """Example 1 (delta = 1/2, C = 1, p^0 = 1): for u = 1 with zero volume constraint,
    L 1(x) = (|B_delta(x) cut by Omega| - pi delta^2)/delta^4; the lattice value converges."""
    errs = []
    for n in (16, 32, 64):
        P = O.Problem(dim=2, n=n, R=n // 2 + 1, kernel="const", norm="none")
        delta = np.full((n, n), 0.5)
        c = np.ones((n, n))
        u = np.ones((n, n))
        got = O.fast_apply_const(P, delta, c, u)
        x = F.nodes(n)
        idx = [(0, 0), (n // 4, n // 2), (n // 2, n // 2), (n - 1, n // 3)]
        e = 0.0
        for i, j in idx:
            ref = (disk_square_area(x[i], x[j], 0.5) - math.pi * 0.25) / 0.5 ** 4
            e = max(e, abs(got[i, j] - ref))
        errs.append(e)
    assert errs[2] < errs[0] / 2.5, errs


# --------------------------------------------------------------- CG
def test_cg_matches_dense_solve():
    n, R = 10, 4
    P = O.Problem(dim=2, n=n, R=R, form="div", kernel="frac")
    delta, c = rand_fields(n, 2, 2.0, 4.0, 31)
    b = np.random.default_rng(32).standard_normal((n, n))
    x, it, rr, ok = O.cg_div(P, delta, c, b, rtol=1e-10)
    assert ok and rr <= 1e-10
    A = -assemble(P, delta, c)
    xd = np.linalg.solve(A, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-8 * np.linalg.norm(xd)


# --------------------------------------------------------------- kernel-averaged form
@pytest.mark.parametrize("dim,n", [(1, 30), (2, 9), (3, 5)])
@pytest.mark.parametrize("kname,kw", [("frac", {"s": 0.5}), ("const", {}), ("inv_r", {})])
def test_sym_is_the_average_of_case_a_and_its_transpose(dim, n, kname, kw):
    """The kernel-averaged operator against the case (a) matrix assembled from
    unit vectors: every in-grid off-diagonal entry is (A_a[i,j] + A_a[j,i]) / 2,
    the diagonal makes every row of the full operator (collar partners
    included) sum to zero, the matrix is symmetric and -A is positive definite
    (Cholesky), and L of a constant is exactly 0."""
    R = 4
    g = np.random.default_rng(60 + dim)
    delta = g.uniform(1.3, 4.0, (n,) * dim) / n
    c = np.exp(g.normal(0.0, 0.5, (n,) * dim))
    Pa = O.Problem(dim=dim, n=n, R=R, form="nd", kernel=kname, **kw)
    Ps = O.Problem(dim=dim, n=n, R=R, form="sym", kernel=kname, **kw)
    Aa = assemble(Pa, delta, c)
    As = assemble(Ps, delta, c)
    N = n ** dim
    off = ~np.eye(N, dtype=bool)
    assert np.allclose(As[off], (0.5 * (Aa + Aa.T))[off], rtol=1e-13, atol=0)
    assert np.abs(As - As.T).max() <= 1e-13 * np.abs(As).max()
    np.linalg.cholesky(-As)
    # the diagonal: minus the in-grid weights minus the collar weights of case (a)
    collar = -Aa.sum(axis=1)  # case (a) rows sum to minus the collar weights
    assert np.allclose(np.diag(As), -(As.sum(axis=1) - np.diag(As)) - collar, rtol=1e-12, atol=0)
    assert np.allclose(O.div_diag(Ps, delta, c).ravel(), -np.diag(As), rtol=1e-12, atol=0)
    u = np.full((n + 2 * R,) * dim, 1.625)
    assert np.all(O.apply(Ps, delta, c, u) == 0.0)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_sym_with_constant_fields_is_case_a(dim):
    """Constant delta and C: both kernels of a pair coincide, so the
    kernel-averaged form is case (a) itself, collar data included."""
    n = {1: 40, 2: 12, 3: 6}[dim]
    R = 5
    delta = np.full((n,) * dim, 3.4 / n)
    c = np.full((n,) * dim, 0.8)
    u = np.random.default_rng(dim).standard_normal((n + 2 * R,) * dim)
    Pa = O.Problem(dim=dim, n=n, R=R, form="nd", kernel="frac")
    Ps = O.Problem(dim=dim, n=n, R=R, form="sym", kernel="frac")
    La, Ls = O.apply(Pa, delta, c, u), O.apply(Ps, delta, c, u)
    assert np.abs(La - Ls).max() <= 1e-13 * np.abs(La).max()
