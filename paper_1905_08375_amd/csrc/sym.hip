// The kernel-averaged symmetric form of the nonlocal diffusion operator:
//
//   L_s u(x) = sum_y w_s(x, y) (u(y) - u(x)) h^d,
//   w_s(x, y) = (omega_x(y) + omega_y(x)) / 2 for y in Omega,  omega_x(y) for y in the collar,
//
// with omega_x(y) = s_x |z|^e on the ball of x (the case (a) weight of Section
// 2, power profiles).  -L_s is SPD, so CG can invert it, and with the pair
// weights split as in Section 3 (m^e plus the remainder) it has a fast
// evaluation: the gather half is the hierarchical path of case (a) itself, and
// the other half is its exact adjoint, a scatter of s_y m_y^e u_y onto the row
// intervals of every ball (difference entries at both ends of each interval)
// followed by prefix sums along the rows.  Written out:
//
//   L_s u = L_a u + (T u - L_a^Omega u) / 2,
//   T u(x)       = sum_{y in Omega} omega_y(x) (u_y - u_x)   (the scatter half),
//   L_a^Omega u  = sum_{y in Omega} omega_x(y) (u_y - u_x)   (the gather half, partners in Omega),
//
// and the fast evaluation forms T u - L_a^Omega u from the scatter, from row
// prefix sums of u with the collar masked, from the per-node sums of both
// weight sets over Omega (set up with the plan), and from the two remainders
// summed directly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace ndl {

// ------------------------------------------------------------------ direct sum
struct SymGeom {
    int ext[3], pext[3], rr[3], H, E[3], L[3], tiles[3];
    int64_t N, NP;
};

static SymGeom sym_geom(const Plan& p, int E0, int E1, int E2)
{
    SymGeom g{};
    const int used[3] = {p.dim >= 3, p.dim >= 2, 1};
    const int E[3] = {E0, E1, E2};
    g.H = p.J;
    for (int a = 0; a < 3; ++a) {
        g.ext[a] = used[a] ? (int)p.n : 1;
        g.pext[a] = used[a] ? (int)p.P : 1;
        g.rr[a] = used[a] ? p.R : 0;
        g.E[a] = used[a] ? E[a] : 1;
        g.L[a] = g.E[a] + (used[a] ? 2 * g.H : 0);
        g.tiles[a] = (g.ext[a] + g.E[a] - 1) / g.E[a];
    }
    g.N = p.N;
    g.NP = p.NP;
    return g;
}

// w_s over the ball of reach J around each node: u of the tile from the
// padded state, the cutoff k and scale s of every node of the tile and its
// halo (k = -1 marks the collar, whose partners keep omega_x).  DIAG: the
// diagonal of -L_s (the sum of the weights) instead of L_s u.
// NPT nodes per thread, E[1] / NPT rows apart (2D: 8 x 64 tiles, so that the
// per-offset work and the halo serve two nodes).
template <typename T, bool DIAG, int NPT>
__global__ __launch_bounds__(256) void k_direct_sym(const T* __restrict__ u, T* __restrict__ out,
                                                    const int32_t* __restrict__ kk, const T* __restrict__ sc,
                                                    const int4* __restrict__ full, const double* __restrict__ fw,
                                                    int nfull, int kmax, SymGeom g)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tot = g.L[0] * g.L[1] * g.L[2];
    T* tu = reinterpret_cast<T*>(smem_raw);
    T* ts = tu + tot;
    int* tk = reinterpret_cast<int*>(ts + tot);
    const int nb = g.tiles[0] * g.tiles[1] * g.tiles[2];
    const int t = xcd_tile(blockIdx.x, nb);
    const int t2 = t % g.tiles[2], t1 = (t / g.tiles[2]) % g.tiles[1], t0 = t / (g.tiles[2] * g.tiles[1]);
    const int org[3] = {t0 * g.E[0], t1 * g.E[1], t2 * g.E[2]};
    const int hal[3] = {g.L[0] > g.E[0] ? g.H : 0, g.L[1] > g.E[1] ? g.H : 0, g.H};
    const T* ub = u + (int64_t)blockIdx.y * g.NP;
    T* ob = out + (int64_t)blockIdx.y * g.N;
    struct Slot {
        T u, s;
        int k;
    };
    int kloc = -1;  // the largest cutoff this thread stages (tile and halo)
    stage_batched(
        tot,
        [&](int idx) {
            const int l2 = idx % g.L[2], rr = idx / g.L[2], l1 = rr % g.L[1], l0 = rr / g.L[1];
            const int x0 = org[0] - hal[0] + l0, x1 = org[1] - hal[1] + l1, x2 = org[2] - hal[2] + l2;
            const bool in = x0 >= 0 && x0 < g.ext[0] && x1 >= 0 && x1 < g.ext[1] && x2 >= 0 && x2 < g.ext[2];
            const int p0 = x0 + g.rr[0], p1 = x1 + g.rr[1], p2 = x2 + g.rr[2];
            const bool pin = p0 >= 0 && p0 < g.pext[0] && p1 >= 0 && p1 < g.pext[1] && p2 >= 0 && p2 < g.pext[2];
            const int64_t gi = ((int64_t)x0 * g.ext[1] + x1) * g.ext[2] + x2;
            Slot v{T(0), T(0), -1};
            if (!DIAG && pin) v.u = ub[((int64_t)p0 * g.pext[1] + p1) * g.pext[2] + p2];
            if (in) {
                v.k = kk[gi];
                v.s = sc[gi];
            }
            return v;
        },
        [&](int idx, const Slot& v) {
            tu[idx] = v.u;
            tk[idx] = v.k;
            ts[idx] = v.s;
            kloc = max(kloc, v.k);
        });
    // the block's largest cutoff: no pair of the tile lies past it (a pair
    // counts if |z|^2 <= k_x or |z|^2 <= k_y, both staged here)
    __shared__ int s_kmax[4];
    kloc = wave_max(kloc);
    if ((threadIdx.x & 63) == 0) s_kmax[threadIdx.x >> 6] = kloc;
    __syncthreads();
    const int kb = min(kmax, max(max(s_kmax[0], s_kmax[1]), max(s_kmax[2], s_kmax[3])));
    const int E1 = g.E[1] / NPT;  // rows of the tile that one pass of the threads covers
    const int e2 = threadIdx.x % g.E[2], e1 = (threadIdx.x / g.E[2]) % E1, e0 = threadIdx.x / (g.E[2] * E1);
    const int x0 = org[0] + e0, x2 = org[2] + e2;
    if (e0 >= g.E[0] || x0 >= g.ext[0] || x2 >= g.ext[2]) return;
    const int ls1 = g.L[2], ls0 = g.L[1] * g.L[2];
    int c[NPT], kx[NPT];
    T sx[NPT], u0[NPT];
    bool valid[NPT];
    Acc<T> acc[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        valid[j] = org[1] + e1 + j * E1 < g.ext[1];
        c[j] = (e0 + hal[0]) * ls0 + (e1 + j * E1 + hal[1]) * ls1 + (e2 + hal[2]);
        kx[j] = tk[c[j]];
        sx[j] = ts[c[j]];
        u0[j] = tu[c[j]];
    }
    for (int q = 0; q < nfull; ++q) {
        const int4 o = full[q];
        if (o.w > kb) break;
        const int off = o.x * ls0 + o.y * ls1 + o.z;
        const T fq = (T)fw[q];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int ky = tk[c[j] + off];
            const T wx = o.w <= kx[j] ? sx[j] : T(0);
            const T wy = ky < 0 ? wx : (o.w <= ky ? ts[c[j] + off] : T(0));  // the collar keeps omega_x
            const T w = T(0.5) * (wx + wy) * fq;
            if (DIAG) acc[j].add_(w);
            else acc[j].fma_(w, tu[c[j] + off] - u0[j]);
        }
        if ((q & 7) == 7) {
#pragma unroll
            for (int j = 0; j < NPT; ++j) acc[j].flush();
        }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        if (!valid[j]) continue;
        const int x1 = org[1] + e1 + j * E1;
        const int64_t gi = ((int64_t)x0 * g.ext[1] + x1) * g.ext[2] + x2;
        ob[gi] = acc[j].value();
    }
}

template <typename T>
static int launch_sym_t(Plan& p, const void* u, void* Lu, int batch, bool diag, hipStream_t s)
{
    int E[3];
    if (p.dim == 1) { E[0] = 1; E[1] = 1; E[2] = 256; }
    else if (p.dim == 2) { E[0] = 1; E[1] = 8; E[2] = 64; }  // two nodes per thread
    else { E[0] = 2; E[1] = 2; E[2] = 64; }
    SymGeom g = sym_geom(p, E[0], E[1], E[2]);
    // two nodes per thread only where the launch still has four blocks per
    // unit: small 2D grids keep one node per thread (twice the blocks)
    bool two = p.dim == 2;
    if (two && (int64_t)g.tiles[1] * g.tiles[2] < 1024) {
        two = false;
        g = sym_geom(p, 1, 4, 64);
    }
    const size_t lds = (size_t)g.L[0] * g.L[1] * g.L[2] * (2 * sizeof(T) + sizeof(int));
    if (lds > 144 * 1024) {
        set_error("kernel-averaged form: horizon too wide for the tile (%zu B of LDS)", lds);
        return NDL_EUNSUPPORTED;
    }
    const void* fn = diag ? (two ? (const void*)k_direct_sym<T, true, 2> : (const void*)k_direct_sym<T, true, 1>)
                          : (two ? (const void*)k_direct_sym<T, false, 2> : (const void*)k_direct_sym<T, false, 1>);
    if (lds > 48 * 1024) NDL_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned nb = (unsigned)(g.tiles[0] * g.tiles[1] * g.tiles[2]);
    auto go = [&](auto npt) {
        constexpr int NPT = decltype(npt)::value;
        if (diag)
            k_direct_sym<T, true, NPT><<<dim3(nb, 1), 256, lds, s>>>(nullptr, static_cast<T*>(Lu), p.d_k,
                                                                    (const T*)p.d_scale, p.d_full,
                                                                    (const double*)p.d_fullw, p.nfull, (int)p.kmax, g);
        else
            k_direct_sym<T, false, NPT><<<dim3(nb, (unsigned)batch), 256, lds, s>>>(
                static_cast<const T*>(u), static_cast<T*>(Lu), p.d_k, (const T*)p.d_scale, p.d_full,
                (const double*)p.d_fullw, p.nfull, (int)p.kmax, g);
    };
    if (two) go(std::integral_constant<int, 2>{});
    else go(std::integral_constant<int, 1>{});
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

int launch_sym(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    return p.prec == NDL_F64 ? launch_sym_t<double>(p, u, Lu, batch, false, s)
                             : launch_sym_t<float>(p, u, Lu, batch, false, s);
}

// ------------------------------------------------------------------ fast evaluation
// Per node, over partners in Omega: the sum of the scatter half's weights
// omega_y(x) and of the gather half's omega_x(y) (set up once per plan).
template <typename T>
__global__ void k_sym_sums(const int32_t* __restrict__ kk, const T* __restrict__ sc, const int4* __restrict__ full,
                           const double* __restrict__ fw, int nfull, int dim, int64_t n, int64_t N,
                           double* __restrict__ sums)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t x[3] = {0, 0, 0}, r = i;
    for (int a = 2; a >= 3 - dim; --a) { x[a] = r % n; r /= n; }
    const int kx = kk[i];
    const double sx = (double)sc[i];
    double col = 0.0, row = 0.0;
    for (int q = 0; q < nfull; ++q) {
        const int4 o = full[q];
        const int64_t y0 = x[0] + o.x, y1 = x[1] + o.y, y2 = x[2] + o.z;
        const bool in = y2 >= 0 && y2 < n && (dim < 2 || (y1 >= 0 && y1 < n)) && (dim < 3 || (y0 >= 0 && y0 < n));
        if (!in) continue;
        const int64_t j = (dim == 3 ? (y0 * n + y1) * n : (dim == 2 ? y1 * n : 0)) + y2;
        if (o.w <= kk[j]) col += (double)sc[j] * fw[q];
        if (o.w <= kx) row += sx * fw[q];
    }
    sums[2 * i] = col;
    sums[2 * i + 1] = row;
}

// Compensated prefix sums along rows (as in the row variant of Step 2):
// out[row][j] = sum_{t < j} in[row][t], j = 0..P, as (hi, lo).  mask_R >= 0:
// entries outside Omega (in padded coordinates) count as zero.
__device__ __forceinline__ void sym_two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <typename TI>
__global__ __launch_bounds__(256) void k_scan_rows(const TI* __restrict__ in, int64_t in_stride,
                                                   double2* __restrict__ out, int64_t P, int64_t nrows, int dim,
                                                   int mask_R, int64_t n)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nrows) return;
    const int lane = threadIdx.x & 63;
    bool row_in = true;
    if (mask_R >= 0) {
        const int64_t r1 = dim >= 2 ? row % P : mask_R, r0 = dim >= 3 ? row / P : mask_R;
        row_in = r1 >= mask_R && r1 < mask_R + n && r0 >= mask_R && r0 < mask_R + n;
    }
    const TI* ir = in + row * in_stride;
    double2* orow = out + row * (P + 1);
    if (lane == 0) orow[0] = make_double2(0.0, 0.0);
    double chi = 0.0, clo = 0.0;
    for (int64_t c0 = 0; c0 < P; c0 += 64) {
        const int64_t j = c0 + lane;
        bool keep = j < P && row_in;
        if (mask_R >= 0) keep = keep && j >= mask_R && j < mask_R + n;
        double hi = keep ? (double)ir[j] : 0.0, lo = 0.0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double ohi = __shfl_up(hi, o, 64), olo = __shfl_up(lo, o, 64);
            if (lane >= o) {
                double s, e;
                sym_two_sum(ohi, hi, s, e);
                hi = s;
                lo = lo + olo + e;
            }
        }
        double s, e;
        sym_two_sum(chi, hi, s, e);
        const double slo = clo + lo + e;
        if (j < P) orow[j + 1] = make_double2(s, slo);
        chi = __shfl(s, 63, 64);
        clo = __shfl(slo, 63, 64);
    }
}

__global__ void k_zero_f64(double* a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// The scatter half's polynomial part: every node y of Omega adds
// v = s_y m_y^e u_y to the row intervals of its ball, as +v at the start and
// -v one past the end of each interval (prefix sums along the rows then give,
// at x, the sum over the y whose ball holds x).
template <typename T, int DIM>
__global__ void k_sym_scatter(const T* __restrict__ u, const int32_t* __restrict__ kk, const T* __restrict__ sc,
                              const T* __restrict__ pw, double* __restrict__ D, int64_t n, int R, int64_t P,
                              int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t x[3] = {0, 0, 0}, r = i;
    for (int a = DIM - 1; a >= 0; --a) { x[a] = r % n + R; r /= n; }
    int64_t pc = 0;
    for (int a = 0; a < DIM; ++a) pc = pc * P + x[a];
    const int k = kk[i];
    const double v = (double)sc[i] * (double)pw[i] * (double)u[pc];
    const int J = (int)sqrt((double)k);
    const int J0 = DIM == 3 ? J : 0, J1 = DIM >= 2 ? J : 0;
    for (int a = -J0; a <= J0; ++a)
        for (int b = -J1; b <= J1; ++b) {
            int rem = k - a * a - b * b;
            if (rem < 0) continue;
            int w = (int)sqrt((double)rem);
            while (w * w > rem) --w;
            while ((w + 1) * (w + 1) <= rem) ++w;
            int64_t row = 0;
            if (DIM == 2) row = x[0] + b;
            if (DIM == 3) row = (x[0] + a) * P + (x[1] + b);
            double* Dr = D + row * (P + 1);
            atomicAdd(Dr + (x[DIM - 1] - w), v);
            atomicAdd(Dr + (x[DIM - 1] + w + 1), -v);
        }
}

struct SymFixArgs {
    int64_t n, P, N, NP;
    int R;
    int kmax, nfull;
};

// L_s u = L_a u + (T u - L_a^Omega u) / 2, added to out (which holds L_a u):
//   T u - L_a^Omega u = [Q(x) - s_x m_x^e G(x)]               polynomial parts
//                     + sum_{y in Omega} (s_y kappa_y(z)[q <= k_y] - s_x kappa_x(z)[q <= k_x]) u_y
//                     - u_x (colsum(x) - rowsum(x)),
// Q the prefix-summed scatter, G the masked row sums over the ball of x.
template <typename T, int DIM, bool KAPPA>
__global__ void k_sym_fix(T* __restrict__ out, const T* __restrict__ u, const int32_t* __restrict__ kk,
                          const T* __restrict__ sc, const T* __restrict__ pw, const double2* __restrict__ SO,
                          const double2* __restrict__ Q, const double* __restrict__ sums,
                          const int4* __restrict__ full, const double* __restrict__ fw, SymFixArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    int64_t g[3] = {0, 0, 0}, xp[3] = {0, 0, 0}, r = i;
    for (int d = DIM - 1; d >= 0; --d) { g[d] = r % a.n; xp[d] = g[d] + a.R; r /= a.n; }
    const int64_t P = a.P;
    int64_t pc = 0, rowc = 0;
    for (int d = 0; d < DIM; ++d) pc = pc * P + xp[d];
    if (DIM == 2) rowc = xp[0];
    if (DIM == 3) rowc = xp[0] * P + xp[1];
    const int k = kk[i];
    const double sx = (double)sc[i], px = (double)pw[i], u0 = (double)u[pc];
    // masked row sums over the ball of x
    const int J = (int)sqrt((double)k);
    const int J0 = DIM == 3 ? J : 0, J1 = DIM >= 2 ? J : 0;
    double ghi = 0.0, glo = 0.0;
    for (int aa = -J0; aa <= J0; ++aa)
        for (int b = -J1; b <= J1; ++b) {
            int rem = k - aa * aa - b * b;
            if (rem < 0) continue;
            int w = (int)sqrt((double)rem);
            while (w * w > rem) --w;
            while ((w + 1) * (w + 1) <= rem) ++w;
            int64_t row = 0;
            if (DIM == 2) row = xp[0] + b;
            if (DIM == 3) row = (xp[0] + aa) * P + (xp[1] + b);
            const double2* Sr = SO + row * (P + 1);
            const double2 hi = Sr[xp[DIM - 1] + w + 1], lo = Sr[xp[DIM - 1] - w];
            ghi += hi.x - lo.x;
            glo += hi.y - lo.y;
        }
    const double2 qv = Q[rowc * (P + 1) + xp[DIM - 1] + 1];
    double corr = (qv.x + qv.y) - sx * px * (ghi + glo);
    if (KAPPA) {
        double kap = 0.0;
        for (int q = 0; q < a.nfull; ++q) {
            const int4 o = full[q];
            if (o.w > a.kmax) break;
            const int64_t y0 = g[0] + (DIM == 3 ? o.x : 0), y1 = g[DIM == 3 ? 1 : 0] + (DIM >= 2 ? o.y : 0);
            const int64_t y2 = g[DIM - 1] + o.z;
            const int64_t yy[3] = {DIM == 3 ? y0 : 0, DIM >= 2 ? y1 : 0, y2};
            bool in = yy[2] >= 0 && yy[2] < a.n;
            if (DIM >= 2) in = in && yy[1] >= 0 && yy[1] < a.n;
            if (DIM >= 3) in = in && yy[0] >= 0 && yy[0] < a.n;
            if (!in) continue;
            const int64_t j = DIM == 3 ? (yy[0] * a.n + yy[1]) * a.n + yy[2] : (DIM == 2 ? yy[1] * a.n + yy[2] : yy[2]);
            const double wz = fw[q];
            const double ay = o.w <= kk[j] ? (double)sc[j] * (wz - (double)pw[j]) : 0.0;
            const double bx = o.w <= k ? sx * (wz - px) : 0.0;
            int64_t pj = 0;
            if (DIM == 1) pj = yy[2] + a.R;
            if (DIM == 2) pj = (yy[1] + a.R) * P + yy[2] + a.R;
            if (DIM == 3) pj = ((yy[0] + a.R) * P + yy[1] + a.R) * P + yy[2] + a.R;
            kap += (ay - bx) * (double)u[pj];
        }
        corr += kap;
    }
    corr -= u0 * (sums[2 * i] - sums[2 * i + 1]);
    out[i] = (T)((double)out[i] + 0.5 * corr);
}

// workspace of the fast form (doubles): masked prefix (2 per entry), scatter
// array (1), its prefix (2), per-node sums (2 per node)
int64_t sym_workspace_elems(const Plan& p)
{
    int64_t rows = 1;
    for (int a = 0; a < p.dim - 1; ++a) rows *= p.P;
    return 5 * rows * (p.P + 1) + 2 * p.N;
}

template <typename T>
static int sym_prepare_t(Plan& p, hipStream_t s)
{
    NDL_HIP(hipMalloc(&p.d_symws, sym_workspace_elems(p) * sizeof(double)));
    double* sums = p.d_symws + (sym_workspace_elems(p) - 2 * p.N);
    k_sym_sums<T><<<(unsigned)((p.N + 255) / 256), 256, 0, s>>>(p.d_k, (const T*)p.d_scale, p.d_full,
                                                              (const double*)p.d_fullw, p.nfull, p.dim, p.n, p.N,
                                                              sums);
    NDL_HIP(hipGetLastError());
    NDL_HIP(hipStreamSynchronize(s));
    return NDL_OK;
}

int sym_prepare(Plan& p, hipStream_t s)
{
    if (p.kernel > NDL_G_FRAC) {
        set_error("kernel-averaged form: power profiles (CONST, INV_R, FRAC) only");
        return NDL_EUNSUPPORTED;
    }
    return p.prec == NDL_F64 ? sym_prepare_t<double>(p, s) : sym_prepare_t<float>(p, s);
}

template <typename T, int DIM>
static int sym_fast_t(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    int64_t rows = 1;
    for (int a = 0; a < DIM - 1; ++a) rows *= p.P;
    double* ws = p.d_symws;
    double2* SO = reinterpret_cast<double2*>(ws);
    double* D = ws + 2 * rows * (p.P + 1);
    double2* Q = reinterpret_cast<double2*>(D + rows * (p.P + 1));
    const double* sums = ws + 5 * rows * (p.P + 1);
    SymFixArgs a{p.n, p.P, p.N, p.NP, p.R, (int)p.kmax, p.nfull};
    const bool kappa = p.kernel != NDL_G_CONST;
    const unsigned nbr = (unsigned)((rows + 3) / 4);
    const unsigned nbn = (unsigned)((p.N + 255) / 256);
    const int64_t dl = rows * (p.P + 1);
    for (int b = 0; b < batch; ++b) {
        const T* ub = static_cast<const T*>(u) + (int64_t)b * p.NP;
        T* ob = static_cast<T*>(Lu) + (int64_t)b * p.N;
        // the gather half with the collar: case (a) through the hierarchical path
        NDL_TRY(launch_fast(p, ub, ob, 1, s));
        k_scan_rows<T><<<nbr, 256, 0, s>>>(ub, p.P, SO, p.P, rows, DIM, p.R, p.n);
        k_zero_f64<<<(unsigned)((dl + 255) / 256), 256, 0, s>>>(D, dl);
        k_sym_scatter<T, DIM><<<nbn, 256, 0, s>>>(ub, p.d_k, (const T*)p.d_scale, (const T*)p.d_split, D, p.n, p.R,
                                                  p.P, p.N);
        k_scan_rows<double><<<nbr, 256, 0, s>>>(D, p.P + 1, Q, p.P, rows, DIM, -1, p.n);
        if (kappa)
            k_sym_fix<T, DIM, true><<<nbn, 256, 0, s>>>(ob, ub, p.d_k, (const T*)p.d_scale, (const T*)p.d_split, SO,
                                                        Q, sums, p.d_full, (const double*)p.d_fullw, a);
        else
            k_sym_fix<T, DIM, false><<<nbn, 256, 0, s>>>(ob, ub, p.d_k, (const T*)p.d_scale, (const T*)p.d_split,
                                                         SO, Q, sums, p.d_full, (const double*)p.d_fullw, a);
        NDL_HIP(hipGetLastError());
    }
    return NDL_OK;
}

int launch_sym_fast(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    if (!p.d_symws) { set_error("plan has no workspace for the fast kernel-averaged form"); return NDL_EINVAL; }
    if (p.prec == NDL_F64) {
        if (p.dim == 1) return sym_fast_t<double, 1>(p, u, Lu, batch, s);
        if (p.dim == 2) return sym_fast_t<double, 2>(p, u, Lu, batch, s);
        return sym_fast_t<double, 3>(p, u, Lu, batch, s);
    }
    if (p.dim == 1) return sym_fast_t<float, 1>(p, u, Lu, batch, s);
    if (p.dim == 2) return sym_fast_t<float, 2>(p, u, Lu, batch, s);
    return sym_fast_t<float, 3>(p, u, Lu, batch, s);
}

// ------------------------------------------------------------------ CG on -L_s
// Jacobi-preconditioned CG for FP64 plans of the kernel-averaged form, one
// problem after another, through ndl_apply (direct) or ndl_apply_fast; FP64
// dot products reduced per block and then in one block (fixed order).
__global__ void k_pad_in(const double* __restrict__ x, double* __restrict__ xp, int dim, int64_t n, int R,
                         int64_t P, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t r = i, pi = 0, mul = 1;
    for (int a = 0; a < dim; ++a) {
        pi += (r % n + R) * mul;
        r /= n;
        mul *= P;
    }
    xp[pi] = x[i];
}

__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* __restrict__ part)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v += a[i] * b[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int np, double* __restrict__ out)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// kind 0: r = b + Lx (A = -L), z = r / d, p = z;  1: x += a p, r += a Lp (A p = -Lp), z = r / d;
// 2: p = z + beta p
__global__ void k_sym_cg_vec(int kind, int64_t n, double a, const double* __restrict__ b, double* __restrict__ x,
                             double* __restrict__ r, double* __restrict__ z, double* __restrict__ p,
                             const double* __restrict__ Lv, const double* __restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (kind == 0) {
        const double ri = b[i] + Lv[i];
        r[i] = ri;
        z[i] = ri / d[i];
        p[i] = ri / d[i];
    } else if (kind == 1) {
        x[i] += a * p[i];
        const double ri = r[i] + a * Lv[i];
        r[i] = ri;
        z[i] = ri / d[i];
    } else {
        p[i] = z[i] + a * p[i];
    }
}

static int sym_cg_one(Plan& p, const double* b, double* x, const ndl_cg_opts* opts, ndl_cg_report* rep,
                      hipStream_t s)
{
    const int64_t N = p.N;
    const bool fast = opts && opts->use_fast;
    if (fast && !p.d_symws) { set_error("use_fast needs a plan made with want_fast"); return NDL_EINVAL; }
    double *xp = nullptr, *Lv = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr, *d = nullptr, *part = nullptr,
           *dot = nullptr;
    NDL_HIP(hipMalloc(&xp, p.NP * sizeof(double)));
    NDL_HIP(hipMalloc(&Lv, N * sizeof(double)));
    NDL_HIP(hipMalloc(&r, N * sizeof(double)));
    NDL_HIP(hipMalloc(&z, N * sizeof(double)));
    NDL_HIP(hipMalloc(&pv, N * sizeof(double)));
    NDL_HIP(hipMalloc(&d, N * sizeof(double)));
    NDL_HIP(hipMalloc(&part, 1024 * sizeof(double)));
    NDL_HIP(hipMalloc(&dot, sizeof(double)));
    std::vector<void*> bufs = {xp, Lv, r, z, pv, d, part, dot};
    auto release = [&]() { for (void* q : bufs) (void)hipFree(q); };
    const unsigned nb = (unsigned)((N + 255) / 256);
    const unsigned nbp = (unsigned)((p.NP + 255) / 256);
    auto apply = [&](const double* v) -> int {
        k_pad_in<<<nb, 256, 0, s>>>(v, xp, p.dim, p.n, p.R, p.P, N);  // the collar stays zero
        return fast ? launch_sym_fast(p, xp, Lv, 1, s) : launch_sym_t<double>(p, xp, Lv, 1, false, s);
    };
    auto dotp = [&](const double* a, const double* c, double* h) -> int {
        k_dot_part<<<1024, 256, 0, s>>>(a, c, N, part);
        k_dot_final<<<1, 256, 0, s>>>(part, 1024, dot);
        NDL_HIP(hipMemcpyAsync(h, dot, sizeof(double), hipMemcpyDeviceToHost, s));
        NDL_HIP(hipStreamSynchronize(s));
        return NDL_OK;
    };
    int rc = NDL_OK;
    auto fail = [&](int e) { release(); return e; };
    k_zero_f64<<<nbp, 256, 0, s>>>(xp, p.NP);
    rc = launch_sym_t<double>(p, nullptr, d, 1, true, s);  // diagonal of -L_s (Jacobi)
    if (rc != NDL_OK) return fail(rc);
    double bb = 0.0;
    if ((rc = dotp(b, b, &bb)) != NDL_OK) return fail(rc);
    if ((rc = apply(x)) != NDL_OK) return fail(rc);
    k_sym_cg_vec<<<nb, 256, 0, s>>>(0, N, 0.0, b, x, r, z, pv, Lv, d);
    double rz = 0.0, rr = 0.0;
    if ((rc = dotp(r, z, &rz)) != NDL_OK) return fail(rc);
    if ((rc = dotp(r, r, &rr)) != NDL_OK) return fail(rc);
    const double rtol = opts && opts->rtol > 0 ? opts->rtol : 1e-8;
    const int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 100000;
    int it = 0;
    const double bn = std::sqrt(bb);
    while (it < max_iter && std::sqrt(rr) > rtol * bn) {
        if ((rc = apply(pv)) != NDL_OK) return fail(rc);
        double pAp = 0.0;
        if ((rc = dotp(pv, Lv, &pAp)) != NDL_OK) return fail(rc);
        pAp = -pAp;
        if (!(pAp > 0.0)) { release(); set_error("CG breakdown (p.Ap <= 0)"); return NDL_EBREAKDOWN; }
        const double alpha = rz / pAp;
        k_sym_cg_vec<<<nb, 256, 0, s>>>(1, N, alpha, b, x, r, z, pv, Lv, d);
        double rz2 = 0.0;
        if ((rc = dotp(r, z, &rz2)) != NDL_OK) return fail(rc);
        if ((rc = dotp(r, r, &rr)) != NDL_OK) return fail(rc);
        k_sym_cg_vec<<<nb, 256, 0, s>>>(2, N, rz2 / rz, b, x, r, z, pv, Lv, d);
        rz = rz2;
        ++it;
    }
    // the true residual with the direct apply
    k_pad_in<<<nb, 256, 0, s>>>(x, xp, p.dim, p.n, p.R, p.P, N);
    if ((rc = launch_sym_t<double>(p, xp, Lv, 1, false, s)) != NDL_OK) return fail(rc);
    k_sym_cg_vec<<<nb, 256, 0, s>>>(0, N, 0.0, b, x, r, z, pv, Lv, d);
    if ((rc = dotp(r, r, &rr)) != NDL_OK) return fail(rc);
    release();
    rep->iters = it;
    rep->outer = 1;
    rep->rel_res_fp64 = bn > 0 ? std::sqrt(rr) / bn : 0.0;
    rep->converged = rep->rel_res_fp64 <= rtol;
    rep->fell_back = 0;
    return rep->converged ? NDL_OK : NDL_ENOCONV;
}

int sym_cg_solve(const ndl_plan* plans, int nprob, const double* const* b, double* const* x,
                 const ndl_cg_opts* opts, ndl_cg_report* reports, hipStream_t s)
{
    int rc_all = NDL_OK;
    for (int i = 0; i < nprob; ++i) {
        Plan& p = *reinterpret_cast<Plan*>(plans[i]);
        if (p.prec != NDL_F64) {
            set_error("CG on the kernel-averaged form runs FP64 plans");
            return NDL_EUNSUPPORTED;
        }
        ndl_cg_report rep{};
        const int rc = sym_cg_one(p, b[i], x[i], opts, &rep, s);
        if (reports) reports[i] = rep;
        if (rc != NDL_OK && rc != NDL_ENOCONV) return rc;
        if (rc == NDL_ENOCONV) rc_all = NDL_ENOCONV;
    }
    return rc_all;
}

}  // namespace ndl
