// Hierarchical evaluation of Section 3 for case (a): nonlocal diffusion and
// linear bond-based peridynamics.
//
//   Step 1  the ball of node x is split into maximal dyadic panels of a tree
//           (Algorithm "recur" with the cube/ball test on node boxes);
//   Step 2  per panel, moments of u about the panel centre, bottom-up (one
//           pass per level, FP64 for every precision): sum_w w^alpha u for the
//           monomials |alpha| <= DEG (DEG = 0 is the paper's partial sum of
//           u; DEG > 0 gives the "sum x^m u" moments that Section 3 asks for
//           polynomials p^{2K} with K > 0, and the peridynamic bond tensor);
//   Step 3  per node, the polynomial part of the kernel summed over the
//           panels of its decomposition from those moments, combined as in
//           eq. "nonlocalP" with the full-ball sum of the same polynomial.
//
// Kernel splitting (the K of Section 3):
//   diffusion, polynomial profile p(r) = sum_j a_j r^2j: exact, no remainder;
//   diffusion, power profile |z|^e: the constant m^e (the value at |z| = m)
//     hierarchically, the remainder kappa(z) = |z|^e - m^e summed directly;
//   peridynamics, pair tensor |z|^(e-2) z z^T: the constant m^(e-2) times
//     z z^T hierarchically (second moments of the displacement per
//     component), the remainder (|z|^(e-2) - m^(e-2)) z z^T summed directly.
// The direct remainder is summed from an LDS tile of u in the same pass.
//
// The tree covers the padded box (grid plus collar), so the decomposition is
// of the whole ball and the collar's volume-constraint data enter exactly as
// in the direct sum; with a zero collar this is the paper's ball cut by Omega.
//
// Step 1 is not stored per node.  On panel rows it has a closed form: on a
// row of scale s (side 2^s nodes) the panels inside the ball are one run
// [lo, hi] of the last-axis index, given by an integer square root of the
// squared radius left after the row's farthest offset; the included panels
// are that run minus the children of the run of inside parents.  The same
// __host__ __device__ routine drives the device gather and the host test hook.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace ndl {

constexpr int kMaxDevices = 64;
constexpr int kMaxLevels = 24;

// ------------------------------------------------------------------ integer helpers
template <typename I>
__host__ __device__ inline I isqrt_i(I v)
{
    if (v < 0) return -1;
    // first guess from a hardware square root (FP32 for 32-bit arguments: an
    // error of a unit or two at most, which the corrections below remove)
    I r = sizeof(I) <= 4 ? (I)sqrtf((float)v) : (I)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// floor and ceiling of v / 2^s (panel sides are powers of two: shifts; the
// arithmetic right shift rounds toward minus infinity)
template <typename I>
__host__ __device__ inline I fshr(I v, int s) { return v >> s; }
template <typename I>
__host__ __device__ inline I cshr(I v, int s) { return -((-v) >> s); }

// farthest squared offset from x to the panel [j a, j a + a - 1] on one axis
template <typename I>
__host__ __device__ inline I far2(I x, I j, I a)
{
    I lo = j * a - x, hi = j * a + a - 1 - x;
    return lo * lo > hi * hi ? lo * lo : hi * hi;
}

// panels of side 2^s on the last axis lying inside {|d| <= isqrt(A)} and inside the domain
template <typename I>
__host__ __device__ inline void inside_run(I x, I A, int s, I E, I& lo, I& hi)
{
    if (A < 0 || E <= 0) { lo = 0; hi = -1; return; }
    I r = isqrt_i<I>(A);
    lo = cshr<I>(x - r, s);
    if (lo < 0) lo = 0;
    hi = fshr<I>(x + r + 1, s) - 1;
    if (hi > E - 1) hi = E - 1;
}

// Largest panel scale that can lie inside a ball of cutoff k in dim dimensions
// (a panel of side a has a corner at offset >= ceil((a-1)/2) on every axis),
// capped at the tree height L.
__host__ __device__ inline int top_scale(int dim, int64_t k, int L)
{
    int s = 0;
    while (s < L) {
        int64_t a = (int64_t)1 << (s + 1);
        int64_t h = a / 2;  // ceil((a-1)/2) for a even
        if ((int64_t)dim * h * h > k) break;
        ++s;
    }
    return s;
}

__host__ __device__ inline int tree_height(int64_t n)
{
    int L = 0;
    while (((int64_t)1 << L) < n) ++L;
    return L;
}

// Step 1 for node x (dim coordinates) in the domain [0, n)^dim, cutoff k:
// calls emit(s, r0, r1, lo, hi) for every run of included panels of scale s
// on the last axis, r0/r1 the row indices on the leading axes (unused axes
// pass 0).  Runs come in increasing s.
template <typename I, class Emit>
__host__ __device__ inline void decompose_runs(int dim, I n, const I* x, I k, Emit& emit)
{
    if (k < 0) return;
    int L = tree_height((int64_t)n);
    int S = top_scale(dim, (int64_t)k, L);
    I J = isqrt_i<I>(k);
    I xl = x[dim - 1];
    for (int s = 0; s <= S; ++s) {
        I a = (I)1 << s;
        I E = n >> s;
        I Ep = n >> (s + 1);
        I rlo[2] = {0, 0}, rhi[2] = {0, 0};
        for (int ax = 0; ax < dim - 1; ++ax) {
            rlo[ax] = cshr<I>(x[ax] - J, s);
            if (rlo[ax] < 0) rlo[ax] = 0;
            rhi[ax] = fshr<I>(x[ax] + J + 1, s) - 1;
            if (rhi[ax] > E - 1) rhi[ax] = E - 1;
        }
        for (I r0 = rlo[0]; r0 <= rhi[0]; ++r0) {
            for (I r1 = rlo[1]; r1 <= rhi[1]; ++r1) {
                I A = k, Ap = k;
                bool prow = s < S;
                if (dim >= 2) {
                    A -= far2<I>(x[0], r0, a);
                    if (prow) { if ((r0 >> 1) > Ep - 1) prow = false; else Ap -= far2<I>(x[0], r0 >> 1, 2 * a); }
                }
                if (dim >= 3) {
                    A -= far2<I>(x[1], r1, a);
                    if (prow) { if ((r1 >> 1) > Ep - 1) prow = false; else Ap -= far2<I>(x[1], r1 >> 1, 2 * a); }
                }
                I lo, hi;
                inside_run<I>(xl, A, s, E, lo, hi);
                if (lo > hi) continue;
                I plo = 0, phi = -1;
                if (prow) inside_run<I>(xl, Ap, s + 1, Ep, plo, phi);
                if (plo > phi) {
                    emit(s, r0, r1, lo, hi);
                } else {
                    if (lo <= 2 * plo - 1) emit(s, r0, r1, lo, 2 * plo - 1);
                    if (2 * phi + 2 <= hi) emit(s, r0, r1, 2 * phi + 2, hi);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ monomials
// Moments are stored per panel as [component][monomial], the monomials
// w0^a0 w1^a1 w2^a2 with a0 + a1 + a2 <= DEG in the order a0, then a1, then a2.
__host__ __device__ constexpr int nmono(int dim, int deg)
{
    return dim == 1 ? deg + 1 : (dim == 2 ? (deg + 1) * (deg + 2) / 2 : (deg + 1) * (deg + 2) * (deg + 3) / 6);
}

template <int DIM, int DEG>
__host__ __device__ constexpr int midx(int a0, int a1, int a2)
{
    if (DIM == 1) return a0;
    if (DIM == 2) return a0 * (DEG + 1) - a0 * (a0 - 1) / 2 + a1;
    int base = 0;
    for (int t = 0; t < a0; ++t) base += nmono(2, DEG - t);
    const int D = DEG - a0;
    return base + a1 * (D + 1) - a1 * (a1 - 1) / 2 + a2;
}

// exponent of axis `ax` of monomial m
template <int DIM, int DEG>
__host__ __device__ constexpr int mexp(int m, int ax)
{
    for (int a0 = 0; a0 <= DEG; ++a0)
        for (int a1 = 0; a1 <= (DIM >= 2 ? DEG - a0 : 0); ++a1)
            for (int a2 = 0; a2 <= (DIM >= 3 ? DEG - a0 - a1 : 0); ++a2)
                if (midx<DIM, DEG>(a0, a1, a2) == m) return ax == 0 ? a0 : (ax == 1 ? a1 : a2);
    return -1;
}

__host__ __device__ constexpr double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

// Moments shifted to a new centre: src holds sum w^b u about centre c, dst
// receives sum (w + d)^alpha u (the same sums about c - d), axis by axis.
template <int DIM, int DEG>
__device__ inline void shift_moments(const double* src, double* dst, const double* d)
{
    constexpr int NM = nmono(DIM, DEG);
    double t[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) t[m] = src[m];
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        double pw[DEG + 1];
        pw[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= DEG; ++q) pw[q] = pw[q - 1] * d[ax];
        double o[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int e0 = mexp<DIM, DEG>(m, 0), e1 = mexp<DIM, DEG>(m, 1), e2 = mexp<DIM, DEG>(m, 2);
            const int ea = ax == 0 ? e0 : (ax == 1 ? e1 : e2);
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b <= DEG; ++b) {
                if (b > ea) break;
                const int src_m = midx<DIM, DEG>(ax == 0 ? b : e0, ax == 1 ? b : e1, ax == 2 ? b : e2);
                acc += binom(ea, b) * pw[ea - b] * t[src_m];
            }
            o[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) t[m] = o[m];
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) dst[m] += t[m];
}

// ------------------------------------------------------------------ Step 2
// Level 1 from the padded state (level 0 is u itself): every node of a panel
// sits at +-1/2 from its centre on each axis.
template <typename T, int DIM, int DEG, int NC>
__global__ __launch_bounds__(256) void k_mom_first(const T* __restrict__ u, int64_t npad, double* __restrict__ lev,
                                                   int64_t P, int64_t E1, int64_t cnt)
{
    constexpr int NM = nmono(DIM, DEG);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int64_t j[3] = {0, 0, 0}, r = t;
    for (int a = DIM - 1; a >= 0; --a) { j[a] = r % E1; r /= E1; }
    double acc[NC * NM];
#pragma unroll
    for (int q = 0; q < NC * NM; ++q) acc[q] = 0.0;
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        int64_t off = 0;
        double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (c >> (DIM - 1 - a)) & 1;
            off = off * P + (2 * j[a] + bit);
            d[a] = bit ? 0.5 : -0.5;
        }
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) {
            const double v = (double)u[comp * npad + off];
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                double w = v;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
#pragma unroll
                    for (int q = 0; q < DEG; ++q)
                        if (q < mexp<DIM, DEG>(m, a)) w *= d[a];
                }
                acc[comp * NM + m] += w;
            }
        }
    }
    double* o = lev + t * (NC * NM);
#pragma unroll
    for (int q = 0; q < NC * NM; ++q) o[q] = acc[q];
}

// Level s from level s-1: the children's moments shifted from their centres to
// the parent's (children sit at +-h, h = a quarter of the parent's side).
template <int DIM, int DEG, int NC>
__global__ __launch_bounds__(256) void k_mom_next(const double* __restrict__ prev, double* __restrict__ lev,
                                                  int64_t Ep, int64_t E, double h, int64_t cnt)
{
    constexpr int NM = nmono(DIM, DEG);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int64_t j[3] = {0, 0, 0}, r = t;
    for (int a = DIM - 1; a >= 0; --a) { j[a] = r % E; r /= E; }
    double acc[NC * NM];
#pragma unroll
    for (int q = 0; q < NC * NM; ++q) acc[q] = 0.0;
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        int64_t off = 0;
        double d[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (c >> (DIM - 1 - a)) & 1;
            off = off * Ep + (2 * j[a] + bit);
            // the child's centre relative to the parent's: w_parent = w_child + d
            d[a] = bit ? h : -h;
        }
        const double* ch = prev + off * (NC * NM);
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) {
            if (DEG == 0) {
                acc[comp] += ch[comp];
            } else {
                double src[NM];
#pragma unroll
                for (int m = 0; m < NM; ++m) src[m] = ch[comp * NM + m];
                shift_moments<DIM, DEG>(src, acc + comp * NM, d);
            }
        }
    }
    double* o = lev + t * (NC * NM);
#pragma unroll
    for (int q = 0; q < NC * NM; ++q) o[q] = acc[q];
}

// ------------------------------------------------------------------ rows (Step 2')
// The row variant of the partial sums: per row of the padded box (all axes
// but the last fixed), compensated prefix sums of u along the row, kept as a
// pair (hi, lo) of FP64 values with hi + lo the exact running sum up to the
// rounding of lo.  S[row][j] = sum_{t < j} u[row][t], j = 0..P; the sum of
// any interval [a, b] is (hi[b+1] - hi[a]) + (lo[b+1] - lo[a]), accurate to
// the interval's own size however far along the row it lies.  One wave per
// row: chunks of 64 values, an inclusive scan across the lanes with exact
// two-sums, and a carry from chunk to chunk.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_row_prefix(const T* __restrict__ u, double2* __restrict__ S, int64_t P,
                                                    int64_t nrows)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nrows) return;
    const int lane = threadIdx.x & 63;
    const T* ur = u + row * P;
    double2* Sr = S + row * (P + 1);
    if (lane == 0) Sr[0] = make_double2(0.0, 0.0);
    double chi = 0.0, clo = 0.0;  // carry: the row's sum so far
    for (int64_t c0 = 0; c0 < P; c0 += 64) {
        const int64_t j = c0 + lane;
        double hi = j < P ? (double)ur[j] : 0.0, lo = 0.0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double ohi = __shfl_up(hi, o, 64), olo = __shfl_up(lo, o, 64);
            if (lane >= o) {
                double s, e;
                two_sum(ohi, hi, s, e);
                hi = s;
                lo = lo + olo + e;
            }
        }
        double s, e;
        two_sum(chi, hi, s, e);
        const double slo = clo + lo + e;
        if (j < P) Sr[j + 1] = make_double2(s, slo);
        chi = __shfl(s, 63, 64);
        clo = __shfl(slo, 63, 64);
    }
}

// ------------------------------------------------------------------ Step 3
struct FastArgs {
    int R, S;
    int poly_mode;              // 1: polynomial profile (weights b_j = a_j / m^2j, no per-node split)
    int P;                      // padded extent per used axis
    int E[3], H, L[3];          // tile extent, LDS halo, LDS extent per box axis
    int tiles[3];
    int ls0, ls1;               // LDS strides of box axes 0, 1
    int ext[3];                 // grid extent per box axis (1 for unused)
    int64_t wrow;               // row length of the full-ball tables (kmax + 1; 1D: isqrt(kmax) + 1)
    int64_t N, NP;
    int64_t lev[kMaxLevels];    // offsets (doubles) of levels 1..S in the pyramid
    double poly[8];             // a_j of the polynomial profile
};

// Polynomial part of one panel for diffusion with p(z) = sum_j b_j |z|^2j:
// sum_{w in Q} p(D + w) u_w from the moments mu of Q (D = panel centre - x).
// The coefficients of p(D + w) in w are built by Horner's rule in
// |D + w|^2 = sum_a (D_a^2 + 2 D_a w_a + w_a^2).
template <int DIM, int DEG>
__device__ inline double panel_poly(const double* mu, const double* D, const double* b)
{
    constexpr int NM = nmono(DIM, DEG);
    constexpr int K = DEG / 2;
    if (K == 0) return b[0] * mu[0];
    double c[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) c[m] = 0.0;
    c[0] = b[K];
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
        double o[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int e[3] = {mexp<DIM, DEG>(m, 0), mexp<DIM, DEG>(m, 1), mexp<DIM, DEG>(m, 2)};
            double acc = m == 0 ? b[j] : 0.0;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                acc += D[ax] * D[ax] * c[m];
                if (e[ax] >= 1) {
                    const int q = midx<DIM, DEG>(e[0] - (ax == 0), e[1] - (ax == 1), e[2] - (ax == 2));
                    acc += 2.0 * D[ax] * c[q];
                }
                if (e[ax] >= 2) {
                    const int q = midx<DIM, DEG>(e[0] - 2 * (ax == 0), e[1] - 2 * (ax == 1), e[2] - 2 * (ax == 2));
                    acc += c[q];
                }
            }
            o[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) c[m] = o[m];
    }
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < NM; ++m) s += c[m] * mu[m];
    return s;
}

// Bond tensor of one panel for peridynamics: F_a += sum_{w in Q} z_a (z . u_w),
// z = D + w, from the moments (|alpha| <= 2) of each displacement component.
template <int DIM>
__device__ inline void panel_pd(const double* mu, const double* D, double* F)
{
    constexpr int NM = nmono(DIM, 2);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double f = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const double* m = mu + b * NM;
            const int eb = midx<DIM, 2>(b == 0, b == 1, b == 2);
            const int ea = midx<DIM, 2>(a == 0, a == 1, a == 2);
            const int eab = midx<DIM, 2>((a == 0) + (b == 0), (a == 1) + (b == 1), (a == 2) + (b == 2));
            f += D[a] * D[b] * m[0] + D[a] * m[eb] + D[b] * m[ea] + m[eab];
        }
        F[a] += f;
    }
}

// MODEL 0 diffusion (NC = 1), 1 peridynamics (NC = DIM).  DEG: moment degree.
// KAPPA: a direct remainder (power profiles).  STAGE: u of the tile plus a halo
// of the ball's reach in LDS (remainder and single-node panels read there).
template <typename T, int DIM, int MODEL, int DEG, bool KAPPA, bool STAGE, int METHOD = 0>
__global__ __launch_bounds__(256) void k_fast_step3(const T* __restrict__ u, T* __restrict__ out,
                                                    const double* __restrict__ pyr, FastArgs a,
                                                    const int32_t* __restrict__ kk, const T* __restrict__ sc,
                                                    const T* __restrict__ pwn, const double* __restrict__ wtab,
                                                    const int4* __restrict__ pairs, const T* __restrict__ pairw,
                                                    int npairs)
{
    constexpr int NC = MODEL ? DIM : 1;
    constexpr int NM = nmono(DIM, DEG);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    __shared__ int64_t s_lev[kMaxLevels];
    constexpr int kStage = 512;
    __shared__ int s_off[KAPPA ? kStage : 1], s_q[KAPPA ? kStage : 1];
    __shared__ T s_w[KAPPA ? kStage : 1];
    __shared__ signed char s_z[KAPPA && MODEL ? 3 * kStage : 1];
    for (int q = threadIdx.x; q < kMaxLevels; q += blockDim.x) s_lev[q] = a.lev[q];
    const bool staged_pairs = KAPPA && STAGE && npairs <= kStage;
    if (staged_pairs)
        for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
            const int4 o = pairs[p];
            s_off[p] = o.x * a.ls0 + o.y * a.ls1 + o.z;
            s_q[p] = o.w;
            s_w[p] = pairw[p];
            if (MODEL) {
                s_z[3 * p] = (signed char)o.x;
                s_z[3 * p + 1] = (signed char)o.y;
                s_z[3 * p + 2] = (signed char)o.z;
            }
        }
    const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
    const int t = xcd_tile(blockIdx.x, nb);
    const int t2 = t % a.tiles[2];
    const int t1 = (t / a.tiles[2]) % a.tiles[1];
    const int t0 = t / (a.tiles[2] * a.tiles[1]);
    const int org[3] = {t0 * a.E[0], t1 * a.E[1], t2 * a.E[2]};
    constexpr bool U0 = DIM >= 3, U1 = DIM >= 2;  // box axes in use
    const int64_t P = a.P;
    const int64_t P0 = U0 ? P : 1, P1 = U1 ? P : 1;
    const T* ub = u + (int64_t)blockIdx.y * NC * a.NP;
    T* ob = out + (int64_t)blockIdx.y * NC * a.N;
    const int tot = a.L[0] * a.L[1] * a.L[2];
    if (STAGE) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            stage_batched(
                tot,
                [&](int idx) {
                    const int l2 = idx % a.L[2];
                    const int rr = idx / a.L[2];
                    const int l1 = rr % a.L[1];
                    const int l0 = rr / a.L[1];
                    // padded coordinates of the staged node
                    const int g0 = U0 ? org[0] + a.R - a.H + l0 : 0;
                    const int g1 = U1 ? org[1] + a.R - a.H + l1 : 0;
                    const int g2 = org[2] + a.R - a.H + l2;
                    const bool in = g0 >= 0 && g0 < P0 && g1 >= 0 && g1 < P1 && g2 >= 0 && g2 < P;
                    const int64_t gg = ((int64_t)g0 * P1 + g1) * P + g2;
                    return in ? ub[c * a.NP + gg] : T(0);
                },
                [&](int idx, T v) { tile[c * tot + idx] = v; });
    }
    __syncthreads();

    const int e2 = threadIdx.x % a.E[2];
    const int e1 = (threadIdx.x / a.E[2]) % a.E[1];
    const int e0 = threadIdx.x / (a.E[2] * a.E[1]);
    const int x[3] = {org[0] + e0, org[1] + e1, org[2] + e2};
    const bool valid = e0 < a.E[0] && x[0] < a.ext[0] && x[1] < a.ext[1] && x[2] < a.ext[2];
    if (!valid) return;
    const int64_t gi = ((int64_t)x[0] * a.ext[1] + x[1]) * a.ext[2] + x[2];
    // this node in the padded box, in the dim coordinates of the tree
    using I = typename std::conditional<DIM == 1, int64_t, int>::type;
    I xp[3] = {0, 0, 0};
    if (DIM == 1) xp[0] = (I)(x[2] + a.R);
    if (DIM == 2) { xp[0] = (I)(x[1] + a.R); xp[1] = (I)(x[2] + a.R); }
    if (DIM == 3) { xp[0] = (I)(x[0] + a.R); xp[1] = (I)(x[1] + a.R); xp[2] = (I)(x[2] + a.R); }
    int64_t pc = 0;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) pc = pc * P + (int64_t)xp[ax];
    const int cidx = STAGE ? (e0 + (U0 ? a.H : 0)) * a.ls0 + (e1 + (U1 ? a.H : 0)) * a.ls1 + (e2 + a.H) : 0;
    auto uval = [&](int c, int64_t gpad, int lidx) -> double {
        return STAGE ? (double)tile[c * tot + lidx] : (double)ub[c * a.NP + gpad];
    };
    double u0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u0[c] = uval(c, pc, cidx);
    const int k = kk[gi];
    // coefficients b_j of the polynomial part in |z|^2j
    double b[DEG / 2 + 1];
    if (MODEL == 0 && a.poly_mode) {
        const double im2 = (double)pwn[gi];
        double pw = 1.0;
#pragma unroll
        for (int j = 0; j <= DEG / 2; ++j) { b[j] = a.poly[j] * pw; pw *= im2; }
    } else {
#pragma unroll
        for (int j = 0; j <= DEG / 2; ++j) b[j] = j == 0 ? 1.0 : 0.0;
    }
    double G[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) G[c] = 0.0;
    // Steps 1 and 3: walk the decomposition, gather the panels
    auto emit = [&](int s, I r0, I r1, I lo, I hi) {
        if (s == 0) {
            // single nodes: the polynomial at the node's own offset
            for (I j = lo; j <= hi; ++j) {
                I y[3] = {0, 0, 0};
                if (DIM == 1) y[0] = j;
                if (DIM == 2) { y[0] = r0; y[1] = j; }
                if (DIM == 3) { y[0] = r0; y[1] = r1; y[2] = j; }
                double z[3] = {0.0, 0.0, 0.0};
                int64_t gpad = 0;
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) {
                    z[ax] = (double)(y[ax] - xp[ax]);
                    gpad = gpad * P + (int64_t)y[ax];
                }
                int lidx = 0;
                if (STAGE) {
                    const int d0 = DIM == 3 ? (int)(y[0] - xp[0]) : 0;
                    const int d1 = DIM >= 2 ? (int)(y[DIM - 2] - xp[DIM - 2]) : 0;
                    const int d2 = (int)(y[DIM - 1] - xp[DIM - 1]);
                    lidx = cidx + d0 * a.ls0 + d1 * a.ls1 + d2;
                }
                if (MODEL == 0) {
                    double w = b[0];
                    if (DEG > 0) {
                        double q2 = 0.0;
#pragma unroll
                        for (int ax = 0; ax < DIM; ++ax) q2 += z[ax] * z[ax];
                        double pw = q2;
#pragma unroll
                        for (int jj = 1; jj <= DEG / 2; ++jj) { w += b[jj] * pw; pw *= q2; }
                    }
                    G[0] += w * uval(0, gpad, lidx);
                } else {
                    double zu = 0.0;
#pragma unroll
                    for (int c = 0; c < NC; ++c) zu += z[c] * uval(c, gpad, lidx);
#pragma unroll
                    for (int c = 0; c < NC; ++c) G[c] += z[c] * zu;
                }
            }
        } else {
            const I side = (I)1 << s;
            const I E = (I)(P >> s);
            const double half = 0.5 * (double)(side - 1);
            double D[3] = {0.0, 0.0, 0.0};
            int64_t row = 0;
            if (DIM == 2) { D[0] = (double)(r0 * side - xp[0]) + half; row = (int64_t)r0 * E; }
            if (DIM == 3) {
                D[0] = (double)(r0 * side - xp[0]) + half;
                D[1] = (double)(r1 * side - xp[1]) + half;
                row = ((int64_t)r0 * E + r1) * E;
            }
            const double* base = pyr + s_lev[s] + row * (NC * NM);
            for (I j = lo; j <= hi; ++j) {
                D[DIM - 1] = (double)(j * side - xp[DIM - 1]) + half;
                const double* mu = base + (int64_t)j * (NC * NM);
                double m[NC * NM];
#pragma unroll
                for (int q = 0; q < NC * NM; ++q) m[q] = mu[q];
                if (MODEL == 0) G[0] += panel_poly<DIM, DEG>(m, D, b);
                else panel_pd<DIM>(m, D, G);
            }
        }
    };
    if (METHOD == 0) {
        decompose_runs<I>(DIM, (I)P, xp, (I)k, emit);
    } else {
        // rows: for every row offset (a, b) of the ball, the interval
        // |z_last| <= isqrt(k - a^2 - b^2) from the row's prefix sums
        const double2* S = reinterpret_cast<const double2*>(pyr);
        const I J = isqrt_i<I>((I)k);
        const I J0 = DIM == 3 ? J : 0, J1 = DIM >= 2 ? J : 0;
        double ghi = 0.0, glo = 0.0;
        // rows in groups of 4: the group's 8 loads are issued before any is
        // used (rows past the ball add exact zeros, the sum order is the rows')
        constexpr int RG = 4;
        for (I a = -J0; a <= J0; ++a)
            for (I b0 = -J1; b0 <= J1; b0 += RG) {
                double2 hv[RG], lv[RG];
#pragma unroll
                for (int i = 0; i < RG; ++i) {
                    const I b2 = b0 + (I)i;
                    const I rem = (I)k - a * a - b2 * b2;
                    hv[i] = make_double2(0.0, 0.0);
                    lv[i] = make_double2(0.0, 0.0);
                    if (b2 <= J1 && rem >= 0) {
                        const I w = isqrt_i<I>(rem);
                        int64_t row = 0;
                        if (DIM == 2) row = (int64_t)(xp[0] + b2);
                        if (DIM == 3) row = (int64_t)(xp[0] + a) * P + (int64_t)(xp[1] + b2);
                        const double2* Sr = S + row * (P + 1);
                        hv[i] = Sr[xp[DIM - 1] + w + 1];
                        lv[i] = Sr[xp[DIM - 1] - w];
                    }
                }
#pragma unroll
                for (int i = 0; i < RG; ++i) {
                    ghi += hv[i].x - lv[i].x;
                    glo += hv[i].y - lv[i].y;
                }
            }
        G[0] = ghi + glo;
    }
    // eq. "nonlocalP": minus the polynomial summed over the full ball times u(x);
    // the tables are indexed by k (1D: by the ball's reach isqrt(k))
    const int64_t kw = DIM == 1 ? (int64_t)isqrt_i<int64_t>((int64_t)k) : (int64_t)k;
    double res[NC];
    const double pw0 = (MODEL == 0 && a.poly_mode) ? 1.0 : (double)pwn[gi];
    if (MODEL == 0) {
        double W = 0.0;
#pragma unroll
        for (int j = 0; j <= DEG / 2; ++j) W += b[j] * wtab[(int64_t)j * a.wrow + kw];
        res[0] = pw0 * (G[0] - W * u0[0]);
    } else {
        const double W = wtab[kw] / (double)DIM;  // sum of z z^T over the ball = T2[k]/dim I
#pragma unroll
        for (int c = 0; c < NC; ++c) res[c] = pw0 * (G[c] - W * u0[c]);
    }
    if (KAPPA) {
        // remainder kappa = w(z) - w(m) over the half ball, pairs {z, -z}
        double kap[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) kap[c] = 0.0;
        for (int p = 0; p < npairs; ++p) {
            int off = 0, q;
            double w;
            int z[3];
            if (staged_pairs) {
                off = s_off[p];
                q = s_q[p];
                w = (double)s_w[p];
                if (MODEL) { z[0] = s_z[3 * p]; z[1] = s_z[3 * p + 1]; z[2] = s_z[3 * p + 2]; }
            } else {
                const int4 o = pairs[p];
                q = o.w;
                w = (double)pairw[p];
                z[0] = o.x; z[1] = o.y; z[2] = o.z;
                off = o.x * a.ls0 + o.y * a.ls1 + o.z;
            }
            if (q > k) break;
            int64_t goff = 0;
            if (!STAGE) goff = ((int64_t)z[0] * P1 + z[1]) * P + z[2];
            const double kwt = w - pw0;
            if (MODEL == 0) {
                const double d = (uval(0, pc + goff, cidx + off) - u0[0]) + (uval(0, pc - goff, cidx - off) - u0[0]);
                kap[0] += kwt * d;
            } else {
                // box axes 3 - DIM .. 2 carry the components 0 .. DIM - 1
                double zc[3] = {0.0, 0.0, 0.0}, proj = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    zc[c] = (double)z[3 - DIM + c];
                    const double d =
                        (uval(c, pc + goff, cidx + off) - u0[c]) + (uval(c, pc - goff, cidx - off) - u0[c]);
                    proj += zc[c] * d;
                }
                proj *= kwt;
#pragma unroll
                for (int c = 0; c < NC; ++c) kap[c] += proj * zc[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) res[c] += kap[c];
    }
    const double s = (double)sc[gi];
#pragma unroll
    for (int c = 0; c < NC; ++c) ob[c * a.N + gi] = (T)(s * res[c]);
}

// Records Step 1 panels for one node on the device (test hook).
struct RecordPanels {
    int dim;
    int32_t* out;
    int cap;
    int count;
    template <typename I>
    __host__ __device__ inline void operator()(int s, I r0, I r1, I lo, I hi)
    {
        for (I j = lo; j <= hi; ++j) {
            if (count < cap) {
                int32_t* rec = out + (size_t)count * (dim + 1);
                rec[0] = s;
                if (dim == 1) rec[1] = (int32_t)j;
                else if (dim == 2) { rec[1] = (int32_t)r0; rec[2] = (int32_t)j; }
                else { rec[1] = (int32_t)r0; rec[2] = (int32_t)r1; rec[3] = (int32_t)j; }
            }
            ++count;
        }
    }
};

__global__ void k_record(int dim, int64_t n, int64_t x0, int64_t x1, int64_t x2, int64_t k, int32_t* out, int cap,
                         int32_t* count)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t x[3] = {x0, x1, x2};
    RecordPanels rp{dim, out, cap, 0};
    decompose_runs<int64_t>(dim, n, x, k, rp);
    *count = rp.count;
}

// ------------------------------------------------------------------ host side
// weight of the polynomial part per node: diffusion m^e, peridynamics m^(e-2)
template <typename T>
__global__ void k_split(const T* __restrict__ delta, int64_t N, int64_t n, double expo, T* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double m = (double)delta[i] * (double)n;
    out[i] = (T)pow(m, expo);
}

// moment degree of a plan's hierarchical path (-1: not supported)
static int fast_degree(const Plan& p)
{
    if (p.kernel == NDL_G_CONE) return -1;  // no polynomial part at the horizon (g(1) = 0)
    if (p.model == NDL_PERIDYNAMIC) return p.kernel == NDL_G_POLY ? -1 : 2;
    if (p.kernel != NDL_G_POLY) return 0;
    const int K = (int)p.poly.size() - 1;
    const int kmax_dim[4] = {0, 3, 2, 1};
    return K <= kmax_dim[p.dim] ? 2 * K : -1;
}

static int fast_ncomp(const Plan& p) { return p.model == NDL_PERIDYNAMIC ? p.dim : 1; }

int fast_prepare(Plan& p, hipStream_t s, bool with_workspace)
{
    if (p.form == NDL_DIV) {
        set_error("the hierarchical path is implemented for case (a) and the kernel-averaged form");
        return NDL_EUNSUPPORTED;
    }
    const int deg = fast_degree(p);
    if (deg < 0) {
        set_error(p.kernel == NDL_G_CONE ? "hierarchical path: the conical profile has no polynomial part"
                  : p.model == NDL_PERIDYNAMIC
                      ? "hierarchical peridynamics needs a power profile"
                      : "hierarchical path: polynomial profiles up to K = 3 (1D), 2 (2D), 1 (3D)");
        return NDL_EUNSUPPORTED;
    }
    if (p.dim >= 2 && p.P > 32767) {
        set_error("hierarchical path: padded extent above 32767");
        return NDL_EUNSUPPORTED;
    }
    p.fast_deg = deg;
    const int nm = nmono(p.dim, deg) * fast_ncomp(p);
    int L = tree_height(p.P);
    p.fast_S = top_scale(p.dim, p.kmax, L);
    if (p.fast_S >= kMaxLevels) { set_error("tree too deep"); return NDL_EUNSUPPORTED; }
    p.lev_off.assign(p.fast_S + 1, 0);
    p.lev_ext.assign(p.fast_S + 1, 0);
    int64_t tot = 0;
    for (int sc = 1; sc <= p.fast_S; ++sc) {
        int64_t E = p.P >> sc;
        int64_t c = 1;
        for (int a = 0; a < p.dim; ++a) c *= E;
        p.lev_off[sc] = tot;
        p.lev_ext[sc] = E;
        tot += c * nm;
    }
    // the row variant (partial sums of degree 0 only) keeps two doubles per
    // prefix entry, (P + 1) entries per row, in the same buffer
    if (deg == 0 && p.model == NDL_DIFFUSION) {
        int64_t rows = 1;
        for (int a = 0; a < p.dim - 1; ++a) rows *= p.P;
        tot = std::max<int64_t>(tot, 2 * rows * (p.P + 1));
    }
    p.pyr_elems = tot;
    if (with_workspace) NDL_HIP(hipMalloc(&p.d_pyr, std::max<int64_t>(1, tot) * sizeof(double)));
    // per-node weight of the polynomial part (power profiles)
    if (p.kernel != NDL_G_POLY) {
        NDL_HIP(hipMalloc(&p.d_split, p.N * elem_size(p.prec)));
        const double e = p.model == NDL_PERIDYNAMIC ? p.expo - 2.0 : p.expo;
        int64_t nb = (p.N + 255) / 256;
        if (p.prec == NDL_F64)
            k_split<double><<<dim3((unsigned)nb), dim3(256), 0, s>>>((const double*)p.prob.delta, p.N, p.n, e,
                                                                    (double*)p.d_split);
        else
            k_split<float><<<dim3((unsigned)nb), dim3(256), 0, s>>>((const float*)p.prob.delta, p.N, p.n, e,
                                                                   (float*)p.d_split);
        NDL_HIP(hipGetLastError());
    }
    // full-ball tables: row j holds sum_{|z|^2 <= k} |z|^2j (centre included)
    // for j = 0..K (diffusion), or the single row sum |z|^2 (peridynamics).
    // In 1D the ball of cutoff k is |z| <= isqrt(k), so the rows are indexed
    // by that reach instead of k.
    std::vector<Off> full = ball_offsets(p.dim, p.kmax, false);
    const int rows = p.model == NDL_PERIDYNAMIC ? 1 : deg / 2 + 1;
    const int64_t wrow = p.dim == 1 ? (int64_t)cisqrt(p.kmax) + 1 : p.kmax + 1;
    std::vector<double> tab((size_t)rows * wrow, 0.0);
    for (int j = 0; j < rows; ++j) {
        const int pw = p.model == NDL_PERIDYNAMIC ? 1 : j;
        std::vector<double> shell(wrow, 0.0);
        if (pw == 0) shell[0] = 1.0;
        for (auto& o : full) shell[p.dim == 1 ? (int64_t)std::abs(o.z0) : o.q] += std::pow((double)o.q, pw);
        double acc = 0.0;
        for (int64_t k = 0; k < wrow; ++k) {
            acc += shell[k];
            tab[(size_t)j * wrow + k] = acc;
        }
    }
    p.fast_wrow = wrow;
    NDL_HIP(hipMalloc(&p.d_wtab, tab.size() * sizeof(double)));
    NDL_HIP(hipMemcpy(p.d_wtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    NDL_HIP(hipStreamSynchronize(s));
    p.fast = true;
    return NDL_OK;
}

static bool fast_has_kappa(const Plan& p)
{
    return !(p.kernel == NDL_G_POLY || (p.kernel == NDL_G_CONST && p.model == NDL_DIFFUSION));
}

// tile of Step 3 (256 nodes) and its LDS halo
static void fast_geometry(const Plan& p, FastArgs& a, bool stage)
{
    int E[3];
    if (p.dim == 1) { E[0] = 1; E[1] = 1; E[2] = 256; }
    else if (p.dim == 2) { E[0] = 1; E[1] = 4; E[2] = 64; }
    else { E[0] = 2; E[1] = 2; E[2] = 64; }
    const int used[3] = {p.dim >= 3, p.dim >= 2, 1};
    a.H = stage ? p.J : 0;
    for (int ax = 0; ax < 3; ++ax) {
        a.E[ax] = E[ax];
        a.ext[ax] = used[ax] ? (int)p.n : 1;
        a.L[ax] = used[ax] ? E[ax] + 2 * a.H : 1;
        a.tiles[ax] = (a.ext[ax] + E[ax] - 1) / E[ax];
    }
    a.ls1 = a.L[2];
    a.ls0 = a.L[1] * a.L[2];
}

static size_t fast_lds(const Plan& p, const FastArgs& a)
{
    return (size_t)a.L[0] * a.L[1] * a.L[2] * fast_ncomp(p) * elem_size(p.prec);
}

// the remainder is staged with the tile when its halo fits the LDS
static bool fast_stage(const Plan& p)
{
    if (!fast_has_kappa(p)) return false;
    FastArgs a{};
    fast_geometry(p, a, true);
    return fast_lds(p, a) <= 96 * 1024;
}

template <typename T, int DIM, int MODEL, int DEG, bool KAPPA, bool STAGE, int METHOD>
static int step3_launch(Plan& p, const FastArgs& a, const T* ub, T* ob, const double* pyr, hipStream_t s)
{
    auto fn = k_fast_step3<T, DIM, MODEL, DEG, KAPPA, STAGE, METHOD>;
    const size_t lds = STAGE ? fast_lds(p, a) : 0;
    if (lds > 48 * 1024)
        NDL_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
    const T* pw = p.kernel == NDL_G_POLY ? (const T*)p.d_invm2 : (const T*)p.d_split;
    fn<<<dim3((unsigned)nb), dim3(256), lds, s>>>(ub, ob, pyr, a, p.d_k, (const T*)p.d_scale, pw, p.d_wtab,
                                                  p.d_pairs, (const T*)p.d_pairw, p.npairs);
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

template <typename T, int DIM, int MODEL, int DEG, int METHOD>
static int step3_dispatch(Plan& p, const FastArgs& a, const T* ub, T* ob, const double* pyr, hipStream_t s)
{
    if (!fast_has_kappa(p)) return step3_launch<T, DIM, MODEL, DEG, false, false, METHOD>(p, a, ub, ob, pyr, s);
    if (a.H > 0) return step3_launch<T, DIM, MODEL, DEG, true, true, METHOD>(p, a, ub, ob, pyr, s);
    return step3_launch<T, DIM, MODEL, DEG, true, false, METHOD>(p, a, ub, ob, pyr, s);
}

template <typename T>
static int rows_launch(Plan& p, const T* ub, double* pyr, hipStream_t s)
{
    int64_t rows = 1;
    for (int a = 0; a < p.dim - 1; ++a) rows *= p.P;
    k_row_prefix<T><<<dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s>>>(ub, reinterpret_cast<double2*>(pyr),
                                                                           p.P, rows);
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

template <typename T, int DIM, int DEG, int NC>
static int step2_launch(Plan& p, const T* ub, double* pyr, hipStream_t s)
{
    for (int sc = 1; sc <= p.fast_S; ++sc) {
        const int64_t E = p.lev_ext[sc];
        int64_t c = 1;
        for (int q = 0; q < DIM; ++q) c *= E;
        if (c == 0) continue;
        const unsigned nb = (unsigned)((c + 255) / 256);
        if (sc == 1)
            k_mom_first<T, DIM, DEG, NC><<<dim3(nb), dim3(256), 0, s>>>(ub, p.NP, pyr + p.lev_off[1], p.P, E, c);
        else
            k_mom_next<DIM, DEG, NC><<<dim3(nb), dim3(256), 0, s>>>(pyr + p.lev_off[sc - 1], pyr + p.lev_off[sc],
                                                                    p.lev_ext[sc - 1], E,
                                                                    0.25 * (double)((int64_t)1 << sc), c);
        NDL_HIP(hipGetLastError());
    }
    return NDL_OK;
}

template <typename T, int DIM, int MODEL, int DEG>
static int launch_fast_k(Plan& p, const void* u, void* Lu, int batch, hipStream_t s, double* pyr)
{
    constexpr int NC = MODEL ? DIM : 1;
    FastArgs a{};
    fast_geometry(p, a, fast_stage(p));
    a.R = p.R;
    a.S = p.fast_S;
    a.poly_mode = p.kernel == NDL_G_POLY ? 1 : 0;
    a.P = (int)std::min<int64_t>(p.P, 0x7fffffff);
    a.wrow = p.fast_wrow;
    a.N = p.N;
    a.NP = p.NP;
    for (int sc = 1; sc <= p.fast_S; ++sc) a.lev[sc] = p.lev_off[sc];
    for (size_t j = 0; j < p.poly.size() && j < 8; ++j) a.poly[j] = p.poly[j];
    for (int b = 0; b < batch; ++b) {
        const T* ub = static_cast<const T*>(u) + (int64_t)b * NC * p.NP;
        T* ob = static_cast<T*>(Lu) + (int64_t)b * NC * p.N;
        if constexpr (MODEL == 0 && DEG == 0) {
            if (p.fast_method == 1) {
                NDL_TRY(rows_launch<T>(p, ub, pyr, s));
                NDL_TRY((step3_dispatch<T, DIM, MODEL, DEG, 1>(p, a, ub, ob, pyr, s)));
                continue;
            }
        }
        NDL_TRY((step2_launch<T, DIM, DEG, NC>(p, ub, pyr, s)));
        NDL_TRY((step3_dispatch<T, DIM, MODEL, DEG, 0>(p, a, ub, ob, pyr, s)));
    }
    return NDL_OK;
}

template <typename T>
static int launch_fast_t(Plan& p, const void* u, void* Lu, int batch, hipStream_t s, double* pyr)
{
    const int d = p.fast_deg;
    if (p.model == NDL_PERIDYNAMIC) {
        if (p.dim == 2) return launch_fast_k<T, 2, 1, 2>(p, u, Lu, batch, s, pyr);
        if (p.dim == 3) return launch_fast_k<T, 3, 1, 2>(p, u, Lu, batch, s, pyr);
    } else if (p.dim == 1) {
        if (d == 0) return launch_fast_k<T, 1, 0, 0>(p, u, Lu, batch, s, pyr);
        if (d == 2) return launch_fast_k<T, 1, 0, 2>(p, u, Lu, batch, s, pyr);
        if (d == 4) return launch_fast_k<T, 1, 0, 4>(p, u, Lu, batch, s, pyr);
        if (d == 6) return launch_fast_k<T, 1, 0, 6>(p, u, Lu, batch, s, pyr);
    } else if (p.dim == 2) {
        if (d == 0) return launch_fast_k<T, 2, 0, 0>(p, u, Lu, batch, s, pyr);
        if (d == 2) return launch_fast_k<T, 2, 0, 2>(p, u, Lu, batch, s, pyr);
        if (d == 4) return launch_fast_k<T, 2, 0, 4>(p, u, Lu, batch, s, pyr);
    } else {
        if (d == 0) return launch_fast_k<T, 3, 0, 0>(p, u, Lu, batch, s, pyr);
        if (d == 2) return launch_fast_k<T, 3, 0, 2>(p, u, Lu, batch, s, pyr);
    }
    set_error("internal: no hierarchical kernel for this plan");
    return NDL_EUNSUPPORTED;
}

int launch_fast(Plan& p, const void* u, void* Lu, int batch, hipStream_t s, double* pyr)
{
    if (!pyr) pyr = p.d_pyr;
    return p.prec == NDL_F64 ? launch_fast_t<double>(p, u, Lu, batch, s, pyr)
                             : launch_fast_t<float>(p, u, Lu, batch, s, pyr);
}

// ------------------------------------------------------------------ static workspace
// The pyramid of ndl_apply_fast_noalloc lives in this file-scope device array
// (each GPU that runs the library holds its own copy until the process ends).
// In host code its name is only a host-side stand-in: the device address of
// each GPU's copy comes from hipGetSymbolAddress, taken once per device with
// that device current and kept here; kernels receive that address.
constexpr int64_t kStaticWorkspaceBytes = int64_t(64) << 20;
static __device__ __align__(256) double scratch[kStaticWorkspaceBytes / sizeof(double)];
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

int fast_static_workspace(double** ptr, int64_t* capacity_elems)
{
    int dev = 0;
    NDL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal %d beyond the static workspace table (%d devices)", dev, kMaxDevices);
        return NDL_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* a = nullptr;
        NDL_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a) { set_error("no device address for the static workspace"); return NDL_EHIP; }
        g_scratch_addr[dev] = a;
    }
    *ptr = static_cast<double*>(g_scratch_addr[dev]);
    *capacity_elems = kStaticWorkspaceBytes / (int64_t)sizeof(double);
    return NDL_OK;
}

int fast_num_methods(const Plan& p) { return p.fast && p.fast_deg == 0 && p.model == NDL_DIFFUSION ? 2 : 1; }

// Device-side record of one node's decomposition (in the tree over the padded
// box: node coordinates shifted by the collar), for the parity test.
int fast_decomp_host(Plan& p, const int64_t* node, int32_t* out, int cap, int* count)
{
    int64_t x[3] = {0, 0, 0};
    for (int a = 0; a < p.dim; ++a) {
        if (node[a] < 0 || node[a] >= p.n) { set_error("node outside the grid"); return NDL_EINVAL; }
        x[a] = node[a] + p.R;
    }
    int64_t gi = 0;
    for (int a = 0; a < p.dim; ++a) gi = gi * p.n + node[a];
    int32_t k = 0;
    NDL_HIP(hipMemcpy(&k, p.d_k + gi, sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t* d_out = nullptr;
    int32_t* d_cnt = nullptr;
    size_t bytes = (size_t)std::max(cap, 1) * (p.dim + 1) * sizeof(int32_t);
    NDL_HIP(hipMalloc(&d_out, bytes));
    NDL_HIP(hipMalloc(&d_cnt, sizeof(int32_t)));
    k_record<<<1, 64>>>(p.dim, p.P, x[0], x[1], x[2], k, d_out, cap, d_cnt);
    NDL_HIP(hipGetLastError());
    int32_t c = 0;
    NDL_HIP(hipMemcpy(&c, d_cnt, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cap > 0)
        NDL_HIP(hipMemcpy(out, d_out, (size_t)std::min(c, cap) * (p.dim + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
    NDL_HIP(hipFree(d_out));
    NDL_HIP(hipFree(d_cnt));
    *count = c;
    return NDL_OK;
}

}  // namespace ndl

// Host evaluation of the same Step 1 routine (no GPU needed).
extern "C" int ndl_decompose_node(int32_t dim, int64_t n, const int64_t* node, int64_t k, int32_t* panels,
                                  int32_t cap, int32_t* count)
{
    using namespace ndl;
    if (dim < 1 || dim > 3 || n < 1 || !node || !count || (cap > 0 && !panels)) {
        set_error("ndl_decompose_node: bad argument");
        return NDL_EINVAL;
    }
    int64_t x[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        if (node[a] < 0 || node[a] >= n) { set_error("node outside the grid"); return NDL_EINVAL; }
        x[a] = node[a];
    }
    RecordPanels rp{dim, panels, cap, 0};
    decompose_runs<int64_t>(dim, n, x, k, rp);
    *count = rp.count;
    return NDL_OK;
}
