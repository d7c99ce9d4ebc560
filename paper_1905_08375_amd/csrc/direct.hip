// Direct quadrature sums of the nonlocal operator (Section 2, eq.
// "eq:diffusion"; linear bond-based peridynamics of Section 1) and the
// per-node set-up they need.
//
// Layout: every problem is handled as a 3-axis box whose leading unused axes
// have extent 1 (1D: 1 x 1 x n, 2D: 1 x n x n).  A block owns a tile of
// E0 x E1 x E2 nodes, stages u (and for case (b) delta, c) for the tile plus a
// halo of H = isqrt(k_max) nodes in LDS, and every thread walks the horizon
// ball of its nodes in order of |z|^2, with a wave-uniform exit once |z|^2
// passes the largest cutoff of the wave.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ndl {

std::vector<Off> ball_offsets(int dim, int64_t kmax, bool half)
{
    int J = cisqrt(kmax);
    std::vector<Off> v;
    int lo1 = dim >= 2 ? -J : 0, hi1 = dim >= 2 ? J : 0;
    int lo2 = dim >= 3 ? -J : 0, hi2 = dim >= 3 ? J : 0;
    for (int a = -J; a <= J; a++)
        for (int b = lo1; b <= hi1; b++)
            for (int c = lo2; c <= hi2; c++) {
                int q = a * a + b * b + c * c;
                if (q == 0 || q > kmax) continue;
                bool pos = a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0)));
                if (half && !pos) continue;
                v.push_back({a, b, c, q});
            }
    std::stable_sort(v.begin(), v.end(), [](const Off& x, const Off& y) { return x.q < y.q; });
    return v;
}

// Map a dim-dimensional offset onto the 3-axis box (leading axes unused).
int4 box_offset(int dim, const Off& o)
{
    if (dim == 1) return make_int4(0, 0, o.z0, o.q);
    if (dim == 2) return make_int4(0, o.z0, o.z1, o.q);
    return make_int4(o.z0, o.z1, o.z2, o.q);
}

// ------------------------------------------------------------------ plan kernels
// k_i = ceil((delta_i n)^2) - 1 in FP64 (the strict lattice ball), plus extremes.
template <typename T>
__global__ __launch_bounds__(256) void k_cutoffs(const T* __restrict__ delta, int64_t N, int64_t n,
                                                 int32_t* __restrict__ kout, int* __restrict__ ext)
{
    __shared__ int smx[4], smn[4];
    int kmx = -1, kmn = 0x7fffffff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double a = (double)delta[i] * (double)n;
        double t = a * a;
        // cutoffs past kMaxCutoff are reported as kMaxCutoff + 1 (the plan rejects them)
        int k = t > (double)kMaxCutoff ? kMaxCutoff + 1 : (int)ceil(t) - 1;
        kout[i] = k;
        kmx = max(kmx, k);
        kmn = min(kmn, k);
    }
    kmx = wave_max(kmx);
    kmn = wave_min(kmn);
    if ((threadIdx.x & 63) == 0) {
        smx[threadIdx.x >> 6] = kmx;
        smn[threadIdx.x >> 6] = kmn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            kmx = max(kmx, smx[w]);
            kmn = min(kmn, smn[w]);
        }
        atomicMax(&ext[0], kmx);
        atomicMin(&ext[1], kmn);
    }
}

// histogram of the integer cutoffs (for the average ball size): per block in
// LDS when the nbins = k_max + 1 bins fit (kKhistLds), then one global add per
// non-empty bin; else straight into the global bins, one add per wave where
// its lanes agree
constexpr int kKhistLds = 4096;
__global__ __launch_bounds__(256) void k_khist(const int32_t* __restrict__ kk, int64_t N, int nbins,
                                               unsigned long long* __restrict__ hist)
{
    extern __shared__ unsigned int sh_hist[];
    const bool in_lds = nbins <= kKhistLds;
    if (in_lds) {
        for (int b = threadIdx.x; b < nbins; b += blockDim.x) sh_hist[b] = 0u;
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int b = kk[i];
        if (in_lds) {
            atomicAdd(&sh_hist[b], 1u);
        } else {
            // a wave whose active lanes share one bin (smooth or constant
            // horizons) adds its count once instead of contending 64 times
            const unsigned long long act = __ballot(1);
            const int lead = __ffsll((unsigned long long)act) - 1;
            const int bl = __shfl(b, lead, 64);
            if (__all(b == bl)) {
                if ((int)(threadIdx.x & 63) == lead) atomicAdd(&hist[b], (unsigned long long)__popcll(act));
            } else {
                atomicAdd(&hist[b], 1ull);
            }
        }
    }
    if (in_lds) {
        __syncthreads();
        for (int b = threadIdx.x; b < nbins; b += blockDim.x)
            if (sh_hist[b]) atomicAdd(&hist[b], (unsigned long long)sh_hist[b]);
    }
}

struct ScaleArgs {
    int dim, kernel, norm, K;
    int64_t n;
    double expo, m2, contc;  // contc = |S^{d-1}| * int_0^1 g(r) r^(d+1) dr
    double poly[8];
};

// Per-node scale s_i of case (a): L u_i = s_i sum_z w(z) (u_{i+z} - u_i), with
// w(z) = |z|^expo for power profiles (s_i = c_i A_i m_i^-expo h^d) and
// w(z) = g(|z|/m_i) for POLY and CONE (s_i = c_i A_i h^d), whose weights the
// kernels form per pair from a per-node value (POLY 1/m_i^2, CONE m_i).
template <typename T>
__global__ void k_scales(const T* __restrict__ delta, const T* __restrict__ coef, const int32_t* __restrict__ kk,
                         int64_t N, ScaleArgs a, const double* __restrict__ Ttab, const int4* __restrict__ full,
                         int nfull, T* __restrict__ sout, T* __restrict__ invm2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double d = (double)delta[i], c = (double)coef[i];
    double nn = (double)a.n;
    double m = d * nn;
    double h = 1.0 / nn, hd = 1.0;
    for (int q = 0; q < a.dim; q++) hd *= h;
    double dd2 = pow(d, (double)(a.dim + 2));
    int k = kk[i];
    double s;
    if (a.kernel <= NDL_G_FRAC) {
        if (a.norm == NDL_NORM_DISCRETE)
            s = Ttab[k] > 0.0 ? c * a.m2 * nn * nn / Ttab[k] : 0.0;
        else if (a.norm == NDL_NORM_CONTINUOUS)
            s = c * a.m2 * pow(m, -a.expo) * hd / (a.contc * dd2);
        else
            s = c * pow(m, -a.expo) * hd / dd2;
    } else {
        // profiles evaluated per pair: POLY p(|z|^2/m^2), CONE (m - |z|)/|z|
        double im2 = 1.0 / (m * m);
        auto gval = [&](int q) {
            if (a.kernel == NDL_G_CONE) return m / sqrt((double)q) - 1.0;
            double r2 = q * im2, pw = 1.0, g = 0.0;
            for (int j = 0; j <= a.K; j++) { g += a.poly[j] * pw; pw *= r2; }
            return g;
        };
        if (a.norm == NDL_NORM_DISCRETE) {
            double tot = 0.0;
            for (int p = 0; p < nfull; p++) {
                int q = full[p].w;
                if (q > k) break;
                tot += gval(q) * q;
            }
            s = tot != 0.0 ? c * a.m2 * nn * nn / tot : 0.0;
        } else if (a.norm == NDL_NORM_CONTINUOUS) {
            s = c * a.m2 * hd / (a.contc * dd2);
        } else {
            s = c * hd / dd2;
        }
        invm2[i] = (T)(a.kernel == NDL_G_CONE ? m : im2);
    }
    sout[i] = (T)s;
}

// ------------------------------------------------------------------ geometry
struct Box {
    int ext[3];     // grid extent per axis (1 for unused)
    int pext[3];    // padded extent per axis
    int rr[3];      // collar per axis
    int halo[3];    // tile halo per axis
    int E[3];       // tile extent per axis
    int L[3];       // LDS extent per axis
    int tiles[3];   // tiles per axis
    int ls0, ls1;   // LDS strides of axes 0 and 1
};

static Box make_box(int dim, int64_t n, int R, int H, int E0, int E1, int E2)
{
    Box b;
    int used[3] = {dim >= 3, dim >= 2, 1};
    int E[3] = {E0, E1, E2};
    for (int a = 0; a < 3; a++) {
        b.ext[a] = used[a] ? (int)n : 1;
        b.pext[a] = used[a] ? (int)(n + 2 * R) : 1;
        b.rr[a] = used[a] ? R : 0;
        b.halo[a] = used[a] ? H : 0;
        b.E[a] = used[a] ? E[a] : 1;
        b.L[a] = b.E[a] + 2 * b.halo[a];
        b.tiles[a] = (b.ext[a] + b.E[a] - 1) / b.E[a];
    }
    b.ls1 = b.L[2];
    b.ls0 = b.L[1] * b.L[2];
    return b;
}

// Stage a tile of the padded field f (plus halo) into LDS; zero outside the box.
template <typename T>
__device__ __forceinline__ void stage(T* __restrict__ lds, const T* __restrict__ f, const Box& B, const int* t0)
{
    int tot = B.L[0] * B.L[1] * B.L[2];
    stage_batched(
        tot,
        [&](int idx) {
            int l2 = idx % B.L[2];
            int r = idx / B.L[2];
            int l1 = r % B.L[1];
            int l0 = r / B.L[1];
            int g0 = t0[0] + B.rr[0] - B.halo[0] + l0;
            int g1 = t0[1] + B.rr[1] - B.halo[1] + l1;
            int g2 = t0[2] + B.rr[2] - B.halo[2] + l2;
            T v = 0;
            if (g0 >= 0 && g0 < B.pext[0] && g1 >= 0 && g1 < B.pext[1] && g2 >= 0 && g2 < B.pext[2])
                v = f[((int64_t)g0 * B.pext[1] + g1) * B.pext[2] + g2];
            return v;
        },
        [&](int idx, T v) { lds[idx] = v; });
}

// ------------------------------------------------------------------ case (a)
// Generic direct sum over the half ball: pairs {z, -z} share |z| and so their
// weight; the second difference (u_+ - u_0) + (u_- - u_0) keeps the
// cancellation exact for smooth u.  NC > 1 is peridynamics with NC = dim
// displacement components (box axes 3 - NC .. 2 carry components 0 .. NC-1):
// the bond projection [z.D] z of the paired second differences D.  PROF: 0
// tabulated power weights, 1 POLY p(|z|^2/m^2), 2 CONE (m - |z|)/|z|, the last
// two formed per pair from the per-node value pv (1/m^2 or m).
template <typename T, int NC, int PROF>
__global__ __launch_bounds__(256) void k_direct_nd(const T* __restrict__ u, T* __restrict__ out,
                                                   const int32_t* __restrict__ kk, const T* __restrict__ sc,
                                                   const T* __restrict__ pv, const int4* __restrict__ pairs,
                                                   const T* __restrict__ pw, int npairs, ScaleArgs a, Box B,
                                                   int64_t N, int64_t NPad, int split)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);
    constexpr bool PD = NC > 1;
    int tot = B.L[0] * B.L[1] * B.L[2];
    // the half-ball table with this tile's flat LDS offsets (uniform reads in the pair loop)
    constexpr int kStage = 512;
    __shared__ int s_off[kStage], s_q[kStage];
    __shared__ short s_z[3][kStage];
    __shared__ T s_w[kStage];
    const bool staged = npairs <= kStage;
    if (staged)
        for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
            int4 o = pairs[p];
            s_off[p] = o.x * B.ls0 + o.y * B.ls1 + o.z;
            s_q[p] = o.w;
            s_z[0][p] = (short)o.x;
            s_z[1][p] = (short)o.y;
            s_z[2][p] = (short)o.z;
            s_w[p] = pw[p];
        }
    int nb = B.tiles[0] * B.tiles[1] * B.tiles[2];
    int t = xcd_tile(blockIdx.x, nb);
    int t2 = t % B.tiles[2];
    int t1 = (t / B.tiles[2]) % B.tiles[1];
    int t0i = t / (B.tiles[2] * B.tiles[1]);
    int org[3] = {t0i * B.E[0], t1 * B.E[1], t2 * B.E[2]};
    const T* ub = u + (int64_t)blockIdx.y * NC * NPad;
    T* ob = out + (int64_t)blockIdx.y * NC * N;
    for (int c = 0; c < NC; c++) stage(tile + c * tot, ub + c * NPad, B, org);
    __syncthreads();

    // `split` lanes (a power of two dividing 64) share one node: lane `sub`
    // takes every split-th pair and the partial sums meet in a shuffle tree
    int npts = B.E[0] * B.E[1] * B.E[2];
    const int sub = threadIdx.x & (split - 1);
    const int pstep = blockDim.x / split;
    for (int pi = threadIdx.x / split; pi < npts; pi += pstep) {
        int e2 = pi % B.E[2];
        int r = pi / B.E[2];
        int e1 = r % B.E[1];
        int e0 = r / B.E[1];
        int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
        bool valid = x0 < B.ext[0] && x1 < B.ext[1] && x2 < B.ext[2];
        int64_t gi = ((int64_t)x0 * B.ext[1] + x1) * B.ext[2] + x2;
        int k = valid ? kk[gi] : -1;
        int kw = wave_max(k);
        int cidx = (e0 + B.halo[0]) * B.ls0 + (e1 + B.halo[1]) * B.ls1 + (e2 + B.halo[2]);
        T u0[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) u0[c] = tile[c * tot + cidx];
        const T pn = PROF != 0 && valid ? pv[gi] : T(0);
        Acc<T> A[NC];
        for (int p = sub, cnt = 0; p < npairs; p += split, cnt++) {
            int zz[3];
            int off, qw;
            T w;
            if (staged) {
                qw = s_q[p];
                off = s_off[p];
                w = s_w[p];
                zz[0] = s_z[0][p]; zz[1] = s_z[1][p]; zz[2] = s_z[2][p];
            } else {
                const int4 o = pairs[p];
                qw = o.w;
                off = o.x * B.ls0 + o.y * B.ls1 + o.z;
                w = pw[p];
                zz[0] = o.x; zz[1] = o.y; zz[2] = o.z;
            }
            if (qw > kw) break;
            if (qw <= k) {
                if (PROF == 1) {
                    T r2 = (T)qw * pn, g = 0, pp = 1;
                    for (int j = 0; j <= a.K; j++) { g += (T)a.poly[j] * pp; pp *= r2; }
                    w = PD ? g / (T)qw : g;
                } else if (PROF == 2) {
                    const T g = pn / sqrt((T)qw) - T(1);
                    w = PD ? g / (T)qw : g;
                }
                if (!PD) {
                    const T d0 = (tile[cidx + off] - u0[0]) + (tile[cidx - off] - u0[0]);
                    A[0].fma_(w, d0);
                } else {
                    T zc[NC], proj = 0;
#pragma unroll
                    for (int c = 0; c < NC; c++) {
                        zc[c] = (T)zz[3 - NC + c];
                        const T d = (tile[c * tot + cidx + off] - u0[c]) + (tile[c * tot + cidx - off] - u0[c]);
                        proj += zc[c] * d;
                    }
                    proj *= w;
#pragma unroll
                    for (int c = 0; c < NC; c++) A[c].fma_(proj, zc[c]);
                }
            }
            if ((cnt & 7) == 7) {
#pragma unroll
                for (int c = 0; c < NC; c++) A[c].flush();
            }
        }
        T v[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) v[c] = A[c].value();
        for (int o = split >> 1; o >= 1; o >>= 1) {
#pragma unroll
            for (int c = 0; c < NC; c++) v[c] += __shfl_xor(v[c], o, 64);
        }
        if (valid && sub == 0) {
            const T s = sc[gi];
#pragma unroll
            for (int c = 0; c < NC; c++) ob[c * N + gi] = s * v[c];
        }
    }
}

// ------------------------------------------------------------------ case (b)
// Symmetric form: each neighbour j uses delta_ij = (delta_i+delta_j)/2 and
// C_ij = (c_i+c_j)/2; k_ij is evaluated in FP64 exactly as in case (a); a
// partner in the collar takes (delta_i, c_i).
struct DivArgs {
    int64_t n;
    int norm, dim;
    double expo, m2, contc, hd;
    int kmax;
};

template <typename T>
__global__ __launch_bounds__(256) void k_direct_div(const T* __restrict__ u, T* __restrict__ out,
                                                    const T* __restrict__ delta, const T* __restrict__ coef,
                                                    const int4* __restrict__ full, const double* __restrict__ fw,
                                                    int nfull, const double* __restrict__ invT, DivArgs a, Box B,
                                                    int64_t N, int64_t NPad, int split)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tu = reinterpret_cast<T*>(smem_raw);
    int nb = B.tiles[0] * B.tiles[1] * B.tiles[2];
    int t = xcd_tile(blockIdx.x, nb);
    int t2 = t % B.tiles[2];
    int t1 = (t / B.tiles[2]) % B.tiles[1];
    int t0i = t / (B.tiles[2] * B.tiles[1]);
    int org[3] = {t0i * B.E[0], t1 * B.E[1], t2 * B.E[2]};
    const T* ub = u + (int64_t)blockIdx.y * NPad;
    T* ob = out + (int64_t)blockIdx.y * N;
    stage(tu, ub, B, org);
    __syncthreads();
    double nn = (double)a.n;
    // `split` lanes share one node as in k_direct_nd; a node's lanes skip or
    // run together, so the shuffle tree below always sees its whole group
    int npts = B.E[0] * B.E[1] * B.E[2];
    const int sub = threadIdx.x & (split - 1);
    const int pstep = blockDim.x / split;
    for (int pi = threadIdx.x / split; pi < npts; pi += pstep) {
        int e2 = pi % B.E[2];
        int r = pi / B.E[2];
        int e1 = r % B.E[1];
        int e0 = r / B.E[1];
        int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
        bool valid = x0 < B.ext[0] && x1 < B.ext[1] && x2 < B.ext[2];
        if (!valid) continue;
        int64_t gi = ((int64_t)x0 * B.ext[1] + x1) * B.ext[2] + x2;
        int cidx = (e0 + B.halo[0]) * B.ls0 + (e1 + B.halo[1]) * B.ls1 + (e2 + B.halo[2]);
        double di = (double)delta[gi], ci = (double)coef[gi];
        T u0 = tu[cidx];
        Acc<T> A0;
        for (int p = sub, cnt = 0; p < nfull; p += split, cnt++) {
            int4 o = full[p];
            if (o.w > a.kmax) break;
            int y0 = x0 + o.x, y1 = x1 + o.y, y2 = x2 + o.z;
            double dj = di, cj = ci;
            if (y0 >= 0 && y0 < B.ext[0] && y1 >= 0 && y1 < B.ext[1] && y2 >= 0 && y2 < B.ext[2]) {
                int64_t gj = ((int64_t)y0 * B.ext[1] + y1) * B.ext[2] + y2;
                dj = (double)delta[gj];
                cj = (double)coef[gj];
            }
            double am = (di + dj) * nn * 0.5;
            double tt = am * am;
            int kij = (int)ceil(tt) - 1;
            if (o.w > kij) continue;
            double C = 0.5 * (ci + cj);
            double w;
            if (a.norm == NDL_NORM_DISCRETE) {
                w = C * fw[p] * invT[kij];
            } else {
                double dij = (di + dj) * 0.5;
                double dd2 = pow(dij, (double)(a.dim + 2));
                double base = C * pow(am, -a.expo) * a.hd / dd2 * fw[p];
                w = a.norm == NDL_NORM_CONTINUOUS ? base * a.m2 / a.contc : base;
            }
            int off = o.x * B.ls0 + o.y * B.ls1 + o.z;
            A0.fma_((T)w, tu[cidx + off] - u0);
            if ((cnt & 7) == 7) A0.flush();
        }
        T v = A0.value();
        for (int o = split >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (sub == 0) ob[gi] = v;
    }
}

// ------------------------------------------------------------------ host side
static double sphere_area(int d) { return d == 1 ? 2.0 : (d == 2 ? 2.0 * M_PI : 4.0 * M_PI); }

static double radial_moment(const Plan& p)
{
    int d = p.dim;
    switch (p.kernel) {
    case NDL_G_CONST: return 1.0 / (d + 2.0);
    case NDL_G_INV_R: return 1.0 / (d + 1.0);
    case NDL_G_FRAC: return 1.0 / (2.0 - 2.0 * p.prob.s);
    case NDL_G_CONE: return 1.0 / (d + 1.0) - 1.0 / (d + 2.0);
    default: {
        double acc = 0.0;
        for (size_t j = 0; j < p.poly.size(); j++) acc += p.poly[j] / (2.0 * j + d + 2.0);
        return acc;
    }
    }
}

static ScaleArgs scale_args(const Plan& p)
{
    ScaleArgs a{};
    a.dim = p.dim;
    a.kernel = p.kernel;
    a.norm = p.norm;
    a.K = (int)p.poly.size() - 1;
    a.n = p.n;
    a.expo = p.expo;
    a.m2 = p.m2;
    a.contc = sphere_area(p.dim) * radial_moment(p);
    for (size_t j = 0; j < p.poly.size() && j < 8; j++) a.poly[j] = p.poly[j];
    return a;
}

// Kernels staging more than 64 KiB of LDS must opt in (gfx950 has 160 KiB per CU).
static int lds_check(const void* fn, size_t lds)
{
    if (lds + 16 * 1024 > 160 * 1024) {
        set_error("kernel tile needs %zu B of LDS (horizon too wide for this tile)", lds);
        return NDL_EUNSUPPORTED;
    }
    // the kernels also hold up to ~16 KiB of static LDS (staged offset tables)
    if (lds + 16 * 1024 > 64 * 1024)
        NDL_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return NDL_OK;
}

template <typename T>
static int upload(void** dst, const std::vector<T>& v)
{
    NDL_HIP(hipMalloc(dst, std::max<size_t>(1, v.size()) * sizeof(T)));
    if (!v.empty()) NDL_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return NDL_OK;
}

template <typename T>
static int plan_fields_t(Plan& p, hipStream_t s)
{
    const T* delta = static_cast<const T*>(p.prob.delta);
    const T* coef = static_cast<const T*>(p.prob.coef);
    int* d_ext = nullptr;
    NDL_HIP(hipMalloc(&d_ext, 2 * sizeof(int)));
    int init[2] = {-1, 0x7fffffff};
    NDL_HIP(hipMemcpyAsync(d_ext, init, sizeof(init), hipMemcpyHostToDevice, s));
    NDL_HIP(hipMalloc(&p.d_k, p.N * sizeof(int32_t)));
    int64_t nblk = (p.N + 255) / 256;
    unsigned ncut = (unsigned)std::min<int64_t>(nblk, 1024);
    k_cutoffs<T><<<dim3(ncut), dim3(256), 0, s>>>(delta, p.N, p.n, p.d_k, d_ext);
    NDL_HIP(hipGetLastError());
    int ext[2];
    NDL_HIP(hipMemcpyAsync(ext, d_ext, sizeof(ext), hipMemcpyDeviceToHost, s));
    NDL_HIP(hipStreamSynchronize(s));
    NDL_HIP(hipFree(d_ext));
    p.kmax = ext[0];
    p.kmin = ext[1];
    if (p.kmax > kMaxCutoff) {
        set_error("horizon too wide: (delta n)^2 above %d somewhere (the per-cutoff tables are bounded)", kMaxCutoff);
        return NDL_EUNSUPPORTED;
    }
    if (p.kmin < 0) {
        set_error("horizon below one grid spacing somewhere (k < 0): delta must be > 0");
        return NDL_EINVAL;
    }
    // the horizon must fit the collar: every |z_a| <= R, i.e. k_max < (R+1)^2
    if (p.kmax > (int64_t)(p.R + 1) * (p.R + 1) - 1) {
        set_error("collar R=%d narrower than the horizon (k_max=%lld needs R >= %d)", p.R,
                  (long long)p.kmax, cisqrt(p.kmax));
        return NDL_EINVAL;
    }
    p.J = cisqrt(p.kmax);
    // offset tables
    std::vector<Off> half = ball_offsets(p.dim, p.kmax, true);
    std::vector<Off> full = ball_offsets(p.dim, p.kmax, false);
    std::vector<int4> hb, fb;
    std::vector<T> hw;
    std::vector<double> fw;
    double e = p.expo;
    for (auto& o : half) {
        hb.push_back(box_offset(p.dim, o));
        double len = std::sqrt((double)o.q);
        double w = std::pow(len, e);
        if (p.model == NDL_PERIDYNAMIC) w /= (double)o.q;
        hw.push_back((T)w);
    }
    for (auto& o : full) {
        fb.push_back(box_offset(p.dim, o));
        fw.push_back(std::pow(std::sqrt((double)o.q), e));
    }
    p.npairs = (int)hb.size();
    p.nfull = (int)fb.size();
    NDL_TRY(upload((void**)&p.d_pairs, hb));
    NDL_TRY(upload(&p.d_pairw, hw));
    if (p.dim == 2 && p.model == NDL_DIFFUSION && p.form == NDL_ND) {
        std::vector<double> wq(p.kmax + 1, 0.0);
        for (int64_t q = 1; q <= p.kmax; ++q) wq[q] = std::pow(std::sqrt((double)q), e);
        NDL_TRY(upload((void**)&p.d_wq, wq));
    }
    NDL_TRY(upload((void**)&p.d_full, fb));
    NDL_TRY(upload(&p.d_fullw, fw));
    // T_e[k] = sum_{0<|z|^2<=k} |z|^(e+2): the discrete second moment up to the m factor
    std::vector<double> Ttab(p.kmax + 1, 0.0);
    {
        std::vector<double> shell(p.kmax + 1, 0.0);
        for (auto& o : full) shell[o.q] += std::pow(std::sqrt((double)o.q), e + 2.0);
        double acc = 0.0;
        for (int64_t k = 0; k <= p.kmax; k++) { acc += shell[k]; Ttab[k] = acc; }
    }
    // case (b): invT[k] = M n^2 / T_e[k]
    std::vector<double> invT(p.kmax + 1, 0.0);
    for (int64_t k = 1; k <= p.kmax; k++) invT[k] = p.m2 * (double)p.n * (double)p.n / Ttab[k];
    NDL_TRY(upload((void**)&p.d_invT, invT));
    double* d_T = nullptr;
    NDL_TRY(upload((void**)&d_T, Ttab));
    // average ball size (neighbours per node) from the histogram of the cutoffs
    {
        std::vector<int64_t> cnt(p.kmax + 1, 0);
        for (auto& o : full) cnt[o.q]++;
        for (int64_t k = 1; k <= p.kmax; k++) cnt[k] += cnt[k - 1];
        unsigned long long* d_hist = nullptr;
        NDL_HIP(hipMalloc(&d_hist, (p.kmax + 1) * sizeof(unsigned long long)));
        NDL_HIP(hipMemsetAsync(d_hist, 0, (p.kmax + 1) * sizeof(unsigned long long), s));
        const int nbins = (int)(p.kmax + 1);
        k_khist<<<dim3(ncut), dim3(256), nbins <= kKhistLds ? nbins * sizeof(unsigned int) : 0, s>>>(p.d_k, p.N,
                                                                                                     nbins, d_hist);
        NDL_HIP(hipGetLastError());
        std::vector<unsigned long long> hist(p.kmax + 1);
        NDL_HIP(hipMemcpyAsync(hist.data(), d_hist, hist.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        NDL_HIP(hipStreamSynchronize(s));
        NDL_HIP(hipFree(d_hist));
        double tot = 0.0;
        for (int64_t k = 0; k <= p.kmax; k++) tot += (double)hist[k] * (double)cnt[k];
        p.avg_ball = p.N > 0 ? tot / (double)p.N : 0.0;
    }
    if (p.form != NDL_DIV) {
        NDL_HIP(hipMalloc(&p.d_scale, p.N * elem_size(p.prec)));
        if (p.kernel == NDL_G_POLY || p.kernel == NDL_G_CONE) NDL_HIP(hipMalloc(&p.d_invm2, p.N * elem_size(p.prec)));
        ScaleArgs a = scale_args(p);
        k_scales<T><<<dim3((unsigned)nblk), dim3(256), 0, s>>>(delta, coef, p.d_k, p.N, a, d_T, p.d_full, p.nfull,
                                                              (T*)p.d_scale, (T*)p.d_invm2);
        NDL_HIP(hipGetLastError());
    }
    NDL_HIP(hipStreamSynchronize(s));
    NDL_HIP(hipFree(d_T));
    return NDL_OK;
}

int plan_fields(Plan& p, hipStream_t s)
{
    return p.prec == NDL_F64 ? plan_fields_t<double>(p, s) : plan_fields_t<float>(p, s);
}

static void default_tile(const Plan& p, int* E)
{
    if (p.tile_x > 0) {
        E[0] = p.tile_z; E[1] = p.tile_y; E[2] = p.tile_x;
        return;
    }
    if (p.dim == 1) { E[0] = 1; E[1] = 1; E[2] = 512; }
    else if (p.dim == 2) { E[0] = 1; E[1] = 16; E[2] = 64; }
    else if (p.model == NDL_PERIDYNAMIC) { E[0] = 2; E[1] = 4; E[2] = 32; }  // three staged components
    else { E[0] = 4; E[1] = 8; E[2] = 32; }
}

// 1D: a few nodes per block would leave most of the chip idle and each thread
// walking the whole ball; small tiles with the pair loop split over 256/E
// lanes per node (a power of two dividing 64) fill the waves instead.
static int tile_and_split(const Plan& p, int* E)
{
    default_tile(p, E);
    if (p.dim != 1) return 1;
    if (p.tile_x <= 0) E[2] = 16;
    return E[2] <= 256 && 256 % E[2] == 0 ? std::min(64, 256 / E[2]) : 1;
}

template <typename T, int NC, int PROF>
static int launch_direct_k(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    int E[3];
    const int split = tile_and_split(p, E);
    Box B = make_box(p.dim, p.n, p.R, p.J, E[0], E[1], E[2]);
    int nb = B.tiles[0] * B.tiles[1] * B.tiles[2];
    size_t lds = (size_t)B.L[0] * B.L[1] * B.L[2] * sizeof(T) * NC;
    NDL_TRY(lds_check((const void*)k_direct_nd<T, NC, PROF>, lds));
    ScaleArgs a = scale_args(p);
    k_direct_nd<T, NC, PROF><<<dim3((unsigned)nb, (unsigned)batch), dim3(256), lds, s>>>(
        static_cast<const T*>(u), static_cast<T*>(Lu), p.d_k, (const T*)p.d_scale, (const T*)p.d_invm2, p.d_pairs,
        (const T*)p.d_pairw, p.npairs, a, B, p.N, p.NP, split);
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

template <typename T, int NC>
static int launch_direct_nc(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    if (p.kernel == NDL_G_POLY) return launch_direct_k<T, NC, 1>(p, u, Lu, batch, s);
    if (p.kernel == NDL_G_CONE) return launch_direct_k<T, NC, 2>(p, u, Lu, batch, s);
    return launch_direct_k<T, NC, 0>(p, u, Lu, batch, s);
}

template <typename T>
static int launch_direct_t(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    if (p.model != NDL_PERIDYNAMIC) return launch_direct_nc<T, 1>(p, u, Lu, batch, s);
    if (p.dim == 2) return launch_direct_nc<T, 2>(p, u, Lu, batch, s);
    return launch_direct_nc<T, 3>(p, u, Lu, batch, s);
}

int launch_direct(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    int rc = launch_direct_2d(p, u, Lu, batch, s);
    if (rc != NDL_EUNSUPPORTED) return rc;
    return p.prec == NDL_F64 ? launch_direct_t<double>(p, u, Lu, batch, s)
                             : launch_direct_t<float>(p, u, Lu, batch, s);
}

template <typename T>
static int launch_div_t(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    int E[3];
    const int split = tile_and_split(p, E);
    Box B = make_box(p.dim, p.n, p.R, p.J, E[0], E[1], E[2]);
    int nb = B.tiles[0] * B.tiles[1] * B.tiles[2];
    size_t lds = (size_t)B.L[0] * B.L[1] * B.L[2] * sizeof(T);
    NDL_TRY(lds_check((const void*)k_direct_div<T>, lds));
    DivArgs a{};
    a.n = p.n;
    a.norm = p.norm;
    a.dim = p.dim;
    a.expo = p.expo;
    a.m2 = p.m2;
    a.contc = sphere_area(p.dim) * radial_moment(p);
    double hd = 1.0;
    for (int q = 0; q < p.dim; q++) hd /= (double)p.n;
    a.hd = hd;
    a.kmax = (int)p.kmax;
    k_direct_div<T><<<dim3((unsigned)nb, (unsigned)batch), dim3(256), lds, s>>>(
        static_cast<const T*>(u), static_cast<T*>(Lu), (const T*)p.prob.delta, (const T*)p.prob.coef, p.d_full,
        (const double*)p.d_fullw, p.nfull, p.d_invT, a, B, p.N, p.NP, split);
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

int launch_div(Plan& p, const void* u, void* Lu, int batch, hipStream_t s)
{
    return p.prec == NDL_F64 ? launch_div_t<double>(p, u, Lu, batch, s)
                             : launch_div_t<float>(p, u, Lu, batch, s);
}

}  // namespace ndl
