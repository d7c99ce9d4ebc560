// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <string>
#include <atomic>
#include <vector>

#include "ndl.h"

namespace ndl {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define NDL_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) return ::ndl::hip_fail(e_, #expr, __FILE__, __LINE__); \
    } while (0)

#define NDL_TRY(expr)                   \
    do {                                \
        int rc_ = (expr);               \
        if (rc_ != NDL_OK) return rc_;  \
    } while (0)

// ------------------------------------------------------------------ lattice
// Largest integer cutoff k = ceil((delta n)^2) - 1 a plan accepts (horizons up
// to 8192 nodes): tables indexed by k stay below 2^26 entries.
constexpr int kMaxCutoff = 1 << 26;

constexpr int cisqrt(int64_t k)
{
    int j = 0;
    while ((int64_t)(j + 1) * (j + 1) <= k) ++j;
    return j;
}

// One offset of the horizon ball: z and q = |z|^2.
struct Off {
    int z0, z1, z2, q;
};

// Offsets z with 0 < |z|^2 <= kmax in `dim` dimensions, sorted by |z|^2 and
// then lexicographically.  half != 0 keeps one of each pair {z, -z} (the one
// whose first non-zero component is positive).
std::vector<Off> ball_offsets(int dim, int64_t kmax, bool half);

// ------------------------------------------------------------------ plan
inline uint64_t next_plan_uid()
{
    static std::atomic<uint64_t> counter{1};
    return counter.fetch_add(1, std::memory_order_relaxed);
}

struct Plan {
    // identity for caches keyed by plan: never reused within a process (a new
    // plan can land at a destroyed plan's address)
    uint64_t uid = next_plan_uid();
    ndl_problem prob{};        // caller's descriptor (poly points at `poly`)
    std::vector<double> poly;  // copied coefficients
    int dim = 0, ncomp = 1, prec = 0, model = 0, form = 0, kernel = 0, norm = 0;
    int64_t n = 0, N = 0;      // nodes per axis, n^dim
    int R = 0;                 // collar
    int64_t P = 0, NP = 0;     // padded extent n + 2R and (n+2R)^dim
    double m2 = 0.0;           // second-moment target
    double expo = 0.0;         // g(|z|/m) = m^-expo |z|^expo for power profiles
    int64_t kmax = 0, kmin = 0;
    int J = 0;                 // isqrt(kmax): reach of the direct sum

    // per-node data (device, owned by the plan)
    int32_t* d_k = nullptr;    // integer cutoff k_i (case (a))
    void* d_scale = nullptr;   // case (a) scale s_i, element type of prec
    void* d_invm2 = nullptr;   // POLY: 1/m_i^2 (element type of prec)
    void* d_split = nullptr;   // fast path: weight of the polynomial part per node
    double* d_invT = nullptr;  // case (b) discrete normalisation 1/T[k], k = 0..kmax

    // half-ball pair table of the generic direct kernel (device, sorted by q)
    int4* d_pairs = nullptr;   // (z0, z1, z2, q)
    void* d_pairw = nullptr;   // weights |z|^expo (diffusion) or |z|^(expo-2) (PD)
    double* d_wq = nullptr;    // |z|^expo by q = |z|^2, q = 0..kmax (2D diffusion, large horizons)
    int npairs = 0;
    int4* d_full = nullptr;    // full ball (case (b))
    void* d_fullw = nullptr;
    int nfull = 0;
    double avg_ball = 0.0;

    // direct-kernel choice
    int variant = 0;
    // block -> tile orders of the specialised 2D kernels for tiles of 8, 16
    // and 32 rows (device), with the tile count each was built for
    int32_t* d_tord[3] = {nullptr, nullptr, nullptr};
    int tord_tiles[3] = {0, 0, 0};
    // largest and smallest cutoff of every 64 x 4 node segment (device)
    int2* d_kseg = nullptr;
    std::vector<double> w2d;   // pair weights of the specialised 2D kernel
    int tile_x = 0, tile_y = 0, tile_z = 0;

    // fast path (Section 3)
    bool fast = false;
    int fast_S = 0;            // largest panel side 2^S used
    int64_t fast_origin = 0;   // tree node index of the first padded node (per axis)
    std::vector<int64_t> lev_off;   // offsets of each level in d_pyr (elements)
    std::vector<int64_t> lev_ext;   // panels per axis on each level
    int fast_deg = 0;          // moment degree of the panels (0: partial sums)
    int fast_method = 0;       // 0: dyadic panels (Steps 1-3), 1: row prefix sums (degree 0 diffusion)
    double* d_pyr = nullptr;   // panel moments, FP64, all levels
    int64_t pyr_elems = 0;
    double* d_symws = nullptr; // workspace of the fast kernel-averaged form
    double* d_wtab = nullptr;  // full-ball sums of the polynomial part per cutoff k
    int64_t fast_wrow = 0;     // row length of d_wtab
};

// host helpers implemented in the .hip files
int plan_fields(Plan& p, hipStream_t s);                   // k_i, scales, tables
int launch_direct(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int launch_div(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
// kernel-averaged symmetric form: direct sum, fast evaluation and its set-up, CG
int launch_sym(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int launch_sym_fast(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int sym_prepare(Plan& p, hipStream_t s);
int sym_cg_solve(const ndl_plan* plans, int nprob, const double* const* b, double* const* x,
                 const ndl_cg_opts* opts, ndl_cg_report* reports, hipStream_t s);
// with_workspace: allocate the plan's own pyramid buffer (ndl_apply_fast);
// without it only ndl_apply_fast_noalloc can run the plan
int fast_prepare(Plan& p, hipStream_t s, bool with_workspace);
// pyr: the pyramid buffer of pyr_elems doubles (nullptr = the plan's own)
int launch_fast(Plan& p, const void* u, void* Lu, int batch, hipStream_t s, double* pyr = nullptr);
// the static pyramid workspace of the calling thread's current device
int fast_static_workspace(double** ptr, int64_t* capacity_elems);
int fast_decomp_host(Plan& p, const int64_t* node, int32_t* out, int cap, int* count);
// 1 if the plan's hierarchical path can run the row variant
int fast_num_methods(const Plan& p);
int autotune(Plan& p, hipStream_t s);
// the direct kernel's tile tuned on the caller's state at the caller's batch
int autotune_apply(Plan& p, const void* u, int batch, hipStream_t s);
// the autotuner's cache (in memory, and the file named by NDL_AUTOTUNE_CACHE)
bool tune_cache_lookup(const std::string& key, int* variant);
void tune_cache_store(const std::string& key, int variant);
bool net_is_linear(void* net);
// z = M(r); add_jacobi (linear mode): z = r dinv + M(r), the two-level form, in the same pass
int net_precond(void* net, const Plan& p, const void* r, void* z, hipStream_t s, const void* dinv = nullptr,
                bool add_jacobi = false);
// Jacobi diagonal inverse of an FP32 case (b) plan's -L (cached with the plan's operator tables)
int plan_dinv_f32(const Plan& P, const float** dinv, hipStream_t s);
int plan_neg_L_f32(const Plan& P, const float* x, float* y, const float** dinv, hipStream_t s);

// element size of a precision
inline size_t elem_size(int prec) { return prec == NDL_F64 ? 8 : 4; }

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Give each XCD a contiguous run of tiles so that neighbouring tiles,
// which share halo rows, hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    int per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// ------------------------------------------------------------------ staging
// Fill the tot slots of an LDS tile: slot idx takes load(idx), written by
// store(idx, value).  Each thread issues the loads of UNR slots before it
// stores any of them, so UNR loads per thread are in flight at once (a loop
// that loads and stores one slot per iteration waits a full memory round
// trip per slot).
template <int UNR = 4, typename F, typename G>
__device__ __forceinline__ void stage_batched(int tot, F&& load, G&& store)
{
    using V = decltype(load(0));
    for (int base = threadIdx.x; base < tot; base += UNR * (int)blockDim.x) {
        V v[UNR];
#pragma unroll
        for (int r = 0; r < UNR; ++r) {
            const int idx = base + r * (int)blockDim.x;
            if (idx < tot) v[r] = load(idx);
        }
#pragma unroll
        for (int r = 0; r < UNR; ++r) {
            const int idx = base + r * (int)blockDim.x;
            if (idx < tot) store(idx, v[r]);
        }
    }
}

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Compensated accumulation: FP64 adds plainly; FP32 keeps a Kahan sum of
// blocks of products (each block a short FMA chain), flushed by the caller.
template <typename T>
struct Acc {
    T sum = 0, comp = 0, blk = 0;
    __device__ __forceinline__ void fma_(T w, T d) { blk = fma(w, d, blk); }
    __device__ __forceinline__ void add_(T v) { blk += v; }
    __device__ __forceinline__ void flush()
    {
        T y = blk - comp;
        T t = sum + y;
        comp = (t - sum) - y;
        sum = t;
        blk = 0;
    }
    __device__ __forceinline__ T value() { flush(); return sum - comp; }
};

template <>
struct Acc<double> {
    double sum = 0;
    __device__ __forceinline__ void fma_(double w, double d) { sum = fma(w, d, sum); }
    __device__ __forceinline__ void add_(double v) { sum += v; }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ double value() { return sum; }
};

int4 box_offset(int dim, const Off& o);
// specialised 2D case (a) diffusion kernel; returns NDL_EUNSUPPORTED when the
// plan is outside its range (the generic kernel then runs)
int launch_direct_2d(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
bool direct_2d_applies(const Plan& p);
int launch_direct_2d_f64(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int launch_direct_2d_f32c(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int launch_direct_2d_f32k(Plan& p, const void* u, void* Lu, int batch, hipStream_t s);
int num_variants_2d();
// plan-time block -> tile orders of the specialised 2D kernels (cost-balanced)
int tile_orders_2d(Plan& p, hipStream_t s);
void variant_tile_2d(const Plan& p, int variant, int* tx, int* ty);
int variant_order_2d(const Plan& p, int variant);

}  // namespace ndl
