// Hierarchical evaluation of Section 3 for case (a) diffusion on the zero
// volume constraint (problem "nonlocal:polynomial"):
//
//   Step 1  the ball of node x cut by Omega is split into maximal dyadic panels
//           of the tree over Omega (Algorithm "recur" with the cube/ball test
//           on node boxes);
//   Step 2  partial sums of u over every panel, bottom-up (one pass per level,
//           FP64 for every precision);
//   Step 3  S_x = sum of the partial sums over the panels of x, and
//           L^P u(x) = s_x w_P (S_x - M_x u(x)) as in eq. "nonlocalP", with
//           M_x the lattice count of the full ball (centre included).
//
// The profile is split as g = kappa + g(1) (the K = 0 splitting): the
// polynomial part is the constant g(1), evaluated hierarchically; the
// remainder kappa(z) = |z|^e - m^e (zero for the constant profile) is summed
// directly in the same kernel.
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

#include "common.h"

namespace ndl {

constexpr int kMaxDevices = 64;

__host__ __device__ inline int64_t isqrt64(int64_t v)
{
    if (v < 0) return -1;
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

__host__ __device__ inline int64_t fdiv(int64_t a, int64_t b)  // floor(a / b), b > 0
{
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b)  // ceil(a / b), b > 0
{
    return -fdiv(-a, b);
}

// floor and ceiling of v / 2^s (panel sides are powers of two: shifts, not
// 64-bit divisions; the arithmetic right shift rounds toward minus infinity)
__host__ __device__ inline int64_t fshr(int64_t v, int s) { return v >> s; }
__host__ __device__ inline int64_t cshr(int64_t v, int s) { return -((-v) >> s); }

// farthest squared offset from x to the panel [j a, j a + a - 1] on one axis
__host__ __device__ inline int64_t far2(int64_t x, int64_t j, int64_t a)
{
    int64_t lo = j * a - x, hi = j * a + a - 1 - x;
    return lo * lo > hi * hi ? lo * lo : hi * hi;
}

// panels of side 2^s on the last axis lying inside {|d| <= isqrt(A)} and inside Omega
__host__ __device__ inline void inside_run(int64_t x, int64_t A, int s, int64_t E, int64_t& lo, int64_t& hi)
{
    if (A < 0 || E <= 0) { lo = 0; hi = -1; return; }
    int64_t r = isqrt64(A);
    lo = cshr(x - r, s);
    if (lo < 0) lo = 0;
    hi = fshr(x + r + 1, s) - 1;
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

// Step 1 for node x (dim coordinates), cutoff k.  Calls
// emit(s, j_rows..., lo, hi) for every run of included panels of scale s on
// the last axis: f(s, r0, r1, lo, hi), where r0/r1 are the row indices on the
// leading axes (unused axes pass 0).
template <class Emit>
__host__ __device__ inline void decompose_runs(int dim, int64_t n, const int64_t* x, int64_t k, Emit& emit)
{
    if (k < 0) return;
    int L = tree_height(n);
    int S = top_scale(dim, k, L);
    int64_t J = isqrt64(k);
    int64_t xl = x[dim - 1];
    for (int s = 0; s <= S; ++s) {
        int64_t a = (int64_t)1 << s;
        int64_t E = n >> s;
        int64_t Ep = n >> (s + 1);
        // row ranges on leading axes
        int64_t rlo[2] = {0, 0}, rhi[2] = {0, 0};
        for (int ax = 0; ax < dim - 1; ++ax) {
            rlo[ax] = cshr(x[ax] - J, s);
            if (rlo[ax] < 0) rlo[ax] = 0;
            rhi[ax] = fshr(x[ax] + J + 1, s) - 1;
            if (rhi[ax] > E - 1) rhi[ax] = E - 1;
        }
        for (int64_t r0 = rlo[0]; r0 <= rhi[0]; ++r0) {
            for (int64_t r1 = rlo[1]; r1 <= rhi[1]; ++r1) {
                int64_t A = k, Ap = k;
                bool prow = s < S;
                if (dim >= 2) {
                    A -= far2(x[0], r0, a);
                    if (prow) { if ((r0 >> 1) > Ep - 1) prow = false; else Ap -= far2(x[0], r0 >> 1, 2 * a); }
                }
                if (dim >= 3) {
                    A -= far2(x[1], r1, a);
                    if (prow) { if ((r1 >> 1) > Ep - 1) prow = false; else Ap -= far2(x[1], r1 >> 1, 2 * a); }
                }
                int64_t lo, hi;
                inside_run(xl, A, s, E, lo, hi);
                if (lo > hi) continue;
                int64_t plo = 0, phi = -1;
                if (prow) inside_run(xl, Ap, s + 1, Ep, plo, phi);
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

// ------------------------------------------------------------------ Step 2
// Level 1 from the padded state (level 0 is u itself), in FP64.
template <typename T>
__global__ void k_pyr_first(const T* __restrict__ u, double* __restrict__ S1, int dim, int64_t n, int R, int64_t E1,
                            int64_t cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int64_t P = n + 2 * R;
    int64_t j[3] = {0, 0, 0}, r = t;
    for (int a = dim - 1; a >= 0; --a) { j[a] = r % E1; r /= E1; }
    double acc = 0.0;
    for (int m = 0; m < (1 << dim); ++m) {
        int64_t off = 0;
        for (int a = 0; a < dim; ++a) off = off * P + (2 * j[a] + ((m >> a) & 1) + R);
        acc += (double)u[off];
    }
    S1[t] = acc;
}

__global__ void k_pyr_next(const double* __restrict__ Sp, double* __restrict__ S, int dim, int64_t Ep, int64_t E,
                           int64_t cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int64_t j[3] = {0, 0, 0}, r = t;
    for (int a = dim - 1; a >= 0; --a) { j[a] = r % E; r /= E; }
    double acc = 0.0;
    for (int m = 0; m < (1 << dim); ++m) {
        int64_t off = 0;
        for (int a = 0; a < dim; ++a) off = off * Ep + (2 * j[a] + ((m >> a) & 1));
        acc += Sp[off];
    }
    S[t] = acc;
}

// ------------------------------------------------------------------ Step 3
struct FastArgs {
    int dim, R, S;
    int64_t n, P;
    int64_t off[24];  // level offsets into the pyramid (levels 1..S)
};

template <typename T>
struct GatherSum {
    const T* u;
    const double* pyr;
    const FastArgs* a;
    double acc;
    __device__ inline void operator()(int s, int64_t r0, int64_t r1, int64_t lo, int64_t hi)
    {
        int dim = a->dim;
        if (s == 0) {
            int64_t base;
            if (dim == 1) base = a->R;
            else if (dim == 2) base = (r0 + a->R) * a->P + a->R;
            else base = ((r0 + a->R) * a->P + (r1 + a->R)) * a->P + a->R;
            for (int64_t j = lo; j <= hi; ++j) acc += (double)u[base + j];
        } else {
            int64_t E = a->n >> s;
            int64_t base = a->off[s];
            if (dim == 2) base += r0 * E;
            else if (dim == 3) base += (r0 * E + r1) * E;
            for (int64_t j = lo; j <= hi; ++j) acc += pyr[base + j];
        }
    }
};

template <typename T, bool KAPPA>
__global__ __launch_bounds__(256) void k_fast_gather(const T* __restrict__ u, T* __restrict__ out,
                                                     const double* __restrict__ pyr, const int32_t* __restrict__ kk,
                                                     const T* __restrict__ sc, const T* __restrict__ split,
                                                     const int32_t* __restrict__ cntM, const int4* __restrict__ pairs,
                                                     const T* __restrict__ pw, int npairs, FastArgs a, int64_t N)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t x[3] = {0, 0, 0}, r = i;
    for (int ax = a.dim - 1; ax >= 0; --ax) { x[ax] = r % a.n; r /= a.n; }
    int64_t pc = 0;
    for (int ax = 0; ax < a.dim; ++ax) pc = pc * a.P + (x[ax] + a.R);
    int k = kk[i];
    GatherSum<T> g{u, pyr, &a, 0.0};
    decompose_runs(a.dim, a.n, x, (int64_t)k, g);
    T u0 = u[pc];
    double wP = (double)split[i];
    double poly = wP * (g.acc - (double)cntM[k] * (double)u0);
    double kap = 0.0;
    if (KAPPA) {
        // remainder kappa(z) = |z|^e - m^e over the ball, paired {z, -z}
        T mp = split[i];
        T sum = 0, comp = 0;
        int64_t s1 = a.dim >= 2 ? a.P : 1;
        int64_t s0 = a.dim >= 3 ? a.P * a.P : 0;
        for (int p = 0; p < npairs; ++p) {
            int4 o = pairs[p];
            if (o.w > k) break;
            int64_t off = (int64_t)o.x * s0 + (int64_t)o.y * s1 + o.z;
            T d = (u[pc + off] - u0) + (u[pc - off] - u0);
            T y = (pw[p] - mp) * d - comp;
            T t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        }
        kap = (double)sum - (double)comp;
    }
    out[i] = (T)((double)sc[i] * (poly + kap));
}

// Records Step 1 panels for one node on the device (test hook).
struct RecordPanels {
    int dim;
    int32_t* out;
    int cap;
    int count;
    __host__ __device__ inline void operator()(int s, int64_t r0, int64_t r1, int64_t lo, int64_t hi)
    {
        for (int64_t j = lo; j <= hi; ++j) {
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
    decompose_runs(dim, n, x, k, rp);
    *count = rp.count;
}

// ------------------------------------------------------------------ host side
template <typename T>
__global__ void k_split(const T* __restrict__ delta, int64_t N, int64_t n, double expo, double a0, T* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double m = (double)delta[i] * (double)n;
    out[i] = (T)(a0 * pow(m, expo));
}

int fast_prepare(Plan& p, hipStream_t s, bool with_workspace)
{
    if (p.kernel == NDL_G_POLY && p.poly.size() > 1) {
        set_error("hierarchical path: polynomial profiles of degree > 0 need panel moments (not built)");
        return NDL_EUNSUPPORTED;
    }
    int L = tree_height(p.n);
    p.fast_S = top_scale(p.dim, p.kmax, L);
    p.lev_off.assign(p.fast_S + 1, 0);
    p.lev_ext.assign(p.fast_S + 1, 0);
    int64_t tot = 0;
    for (int sc = 1; sc <= p.fast_S; ++sc) {
        int64_t E = p.n >> sc;
        int64_t c = 1;
        for (int a = 0; a < p.dim; ++a) c *= E;
        p.lev_off[sc] = tot;
        p.lev_ext[sc] = E;
        tot += c;
    }
    if (p.fast_S > 23) { set_error("tree too deep"); return NDL_EUNSUPPORTED; }
    p.pyr_elems = tot;
    if (with_workspace) NDL_HIP(hipMalloc(&p.d_pyr, std::max<int64_t>(1, tot) * sizeof(double)));
    // weight of the polynomial part per node: g(1) in units of the scale, m^e
    NDL_HIP(hipMalloc(&p.d_split, p.N * elem_size(p.prec)));
    double a0 = p.kernel == NDL_G_POLY ? p.poly[0] : 1.0;
    double e = p.kernel == NDL_G_POLY ? 0.0 : p.expo;
    int64_t nb = (p.N + 255) / 256;
    if (p.prec == NDL_F64)
        k_split<double><<<dim3((unsigned)nb), dim3(256), 0, s>>>((const double*)p.prob.delta, p.N, p.n, e, a0,
                                                                (double*)p.d_split);
    else
        k_split<float><<<dim3((unsigned)nb), dim3(256), 0, s>>>((const float*)p.prob.delta, p.N, p.n, e, a0,
                                                               (float*)p.d_split);
    NDL_HIP(hipGetLastError());
    // M(k) = number of lattice points with |z|^2 <= k, centre included
    std::vector<Off> full = ball_offsets(p.dim, p.kmax, false);
    std::vector<int32_t> cnt(p.kmax + 1, 0);
    for (auto& o : full) cnt[o.q]++;
    cnt[0] += 1;
    for (int64_t k = 1; k <= p.kmax; ++k) cnt[k] += cnt[k - 1];
    NDL_HIP(hipMalloc(&p.d_cntM, cnt.size() * sizeof(int32_t)));
    NDL_HIP(hipMemcpy(p.d_cntM, cnt.data(), cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    NDL_HIP(hipStreamSynchronize(s));
    p.fast = true;
    return NDL_OK;
}

template <typename T>
static int launch_fast_t(Plan& p, const void* u, void* Lu, int batch, hipStream_t s, double* pyr)
{
    FastArgs a{};
    a.dim = p.dim;
    a.R = p.R;
    a.S = p.fast_S;
    a.n = p.n;
    a.P = p.P;
    for (int sc = 1; sc <= p.fast_S; ++sc) a.off[sc] = p.lev_off[sc];
    bool kappa = !(p.kernel == NDL_G_CONST || p.kernel == NDL_G_POLY);
    for (int b = 0; b < batch; ++b) {
        const T* ub = static_cast<const T*>(u) + (int64_t)b * p.NP;
        T* ob = static_cast<T*>(Lu) + (int64_t)b * p.N;
        for (int sc = 1; sc <= p.fast_S; ++sc) {
            int64_t E = p.lev_ext[sc];
            int64_t c = 1;
            for (int q = 0; q < p.dim; ++q) c *= E;
            if (c == 0) continue;
            unsigned nb = (unsigned)((c + 255) / 256);
            if (sc == 1)
                k_pyr_first<T><<<dim3(nb), dim3(256), 0, s>>>(ub, pyr + p.lev_off[1], p.dim, p.n, p.R, E, c);
            else
                k_pyr_next<<<dim3(nb), dim3(256), 0, s>>>(pyr + p.lev_off[sc - 1], pyr + p.lev_off[sc],
                                                          p.dim, p.lev_ext[sc - 1], E, c);
            NDL_HIP(hipGetLastError());
        }
        unsigned nb = (unsigned)((p.N + 255) / 256);
        if (kappa)
            k_fast_gather<T, true><<<dim3(nb), dim3(256), 0, s>>>(ub, ob, pyr, p.d_k, (const T*)p.d_scale,
                                                                 (const T*)p.d_split, p.d_cntM,
                                                                 p.d_pairs, (const T*)p.d_pairw, p.npairs, a, p.N);
        else
            k_fast_gather<T, false><<<dim3(nb), dim3(256), 0, s>>>(ub, ob, pyr, p.d_k, (const T*)p.d_scale,
                                                                  (const T*)p.d_split, p.d_cntM,
                                                                  p.d_pairs, (const T*)p.d_pairw, p.npairs, a, p.N);
        NDL_HIP(hipGetLastError());
    }
    return NDL_OK;
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

// Device-side record of one node's decomposition, for the parity test.
int fast_decomp_host(Plan& p, const int64_t* node, int32_t* out, int cap, int* count)
{
    int64_t x[3] = {0, 0, 0};
    for (int a = 0; a < p.dim; ++a) {
        if (node[a] < 0 || node[a] >= p.n) { set_error("node outside the grid"); return NDL_EINVAL; }
        x[a] = node[a];
    }
    int64_t gi = 0;
    for (int a = 0; a < p.dim; ++a) gi = gi * p.n + x[a];
    int32_t k = 0;
    NDL_HIP(hipMemcpy(&k, p.d_k + gi, sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t* d_out = nullptr;
    int32_t* d_cnt = nullptr;
    size_t bytes = (size_t)std::max(cap, 1) * (p.dim + 1) * sizeof(int32_t);
    NDL_HIP(hipMalloc(&d_out, bytes));
    NDL_HIP(hipMalloc(&d_cnt, sizeof(int32_t)));
    k_record<<<1, 64>>>(p.dim, p.n, x[0], x[1], x[2], k, d_out, cap, d_cnt);
    NDL_HIP(hipGetLastError());
    int32_t c = 0;
    NDL_HIP(hipMemcpy(&c, d_cnt, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cap > 0) NDL_HIP(hipMemcpy(out, d_out, (size_t)std::min(c, cap) * (p.dim + 1) * sizeof(int32_t),
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
    decompose_runs(dim, n, x, k, rp);
    *count = rp.count;
    return NDL_OK;
}
