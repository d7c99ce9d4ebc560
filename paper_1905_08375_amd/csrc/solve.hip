// Batched (Jacobi-)preconditioned CG on -L x = b for case (b) operators
// (the symmetric form of Section 2), used as a Krylov solver around the
// nonlocal matvec as the paper's conclusion proposes.
//
// Many independent problems with uneven grids run together: all vectors of
// all problems live in one concatenated buffer per kind, and every kernel
// walks one table of work items (problem, tile of 64 x 16 nodes in 2D or
// 32 x 8 x 4 in 3D).  Per-item partial dot products are reduced per problem
// in a fixed order (deterministic FP64 sums), per-problem scalars and
// convergence flags stay on the device, and converged problems skip their
// items.  The inner iterations are captured once as a HIP graph of G
// iterations and replayed; the host reads one flag block per replay.
//
// Precision: FP64 plans run plain FP64 CG.  FP32 plans run an FP64 iterative
// refinement: the true residual r = b + L x is formed with an FP64 apply of
// the same operator, the inner FP32 CG solves -L d = r / ||r|| to a relative
// tolerance, and x += ||r|| d in FP64; every dot product and norm is FP64.
#include <algorithm>
#include <chrono>
#include <string>
#include <cmath>
#include <memory>
#include <type_traits>

#include "common.h"

namespace ndl {

// ------------------------------------------------------------------ batched layout
struct Inst {
    int dim, n, J, kmax;
    int nq;                  // ball offsets with |z|^2 <= kmax (prefix of the shared table)
    int tiles[3];
    int E[3];
    int64_t N, off;          // points and offset into the concatenated vectors
    int item0, nitems;       // items of this problem
    const void* delta;       // per-node horizon (element type of the vectors)
    const void* coef;
    double n2;               // n^2
    int norm;                // normalisation mode
    int wtab;                // the batch's kmax < w2_width(dim, J): the shell-weight table follows Tinv
    double expo, m2, contc, hd;
};

// Per-problem scalars (device)
struct Scal {
    double rz, rz_new, pq, rr, alpha, beta, bnorm2, tol2;
    int done, iters, pad0, pad1;
};

static __device__ __forceinline__ int stage_box_len(const int* L) { return L[0] * L[1] * L[2]; }

// One item = one tile of one problem.  The state is read unpadded with zero
// outside Omega (the zero volume constraint of the solve).
template <typename T>
__device__ __forceinline__ void item_geom(const Inst& I, int tile, int* org)
{
    int t2 = tile % I.tiles[2];
    int t1 = (tile / I.tiles[2]) % I.tiles[1];
    int t0 = tile / (I.tiles[2] * I.tiles[1]);
    org[0] = t0 * I.E[0];
    org[1] = t1 * I.E[1];
    org[2] = t2 * I.E[2];
}

__device__ __forceinline__ double block_sum(double v, double* red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;  // valid in thread 0
}

// q = -L p over the items (case (b), FP64 pair cutoffs), fused with the
// per-item partial of p.q.  DIAG = true computes the Jacobi diagonal instead.
// The tile of p and, for FP32 data, of delta and c (with a halo of J nodes)
// are staged in LDS; outside Omega delta is marked negative so a partner in
// the collar takes (delta_i, c_i).  Per pair, in FP64:
//   a = (delta_i + delta_j) (n/2),  k_ij = ceil(a*a) - 1  (exactly the rule of case (b)),
//   w = (c'_i + c'_j) |z|^e M / T_e[k_ij],  c' = c n^2 / 2.
constexpr int kMaxOffs = 512;  // ball offsets staged per item (|z|^2 <= kmax)
// Shell-weight table of the batch's balls, stored after the normalisation
// table at kW2Off with rows of w2_width(dim, J) entries (J the batch's reach,
// so k_ij <= J^2 - 1 stays within a row): W[s][k] = |z|^e M / T_e[k] for the
// shell |z|^2 = s when s <= k, else 0.  One lookup at (|z|^2, k_ij) gives the
// ball test and both factors of the pair weight.
constexpr int kW2Off = 256;
__host__ __device__ constexpr int w2_width(int dim, int J) { return dim == 3 ? 16 : J * J; }

template <typename T, bool DIAG, bool DISC>
__global__ __launch_bounds__(256) void k_div_items(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                   int nitems, const T* __restrict__ pvec, T* __restrict__ qvec,
                                                   const int4* __restrict__ full, const double* __restrict__ fw,
                                                   int nfull, const double* __restrict__ Tinv,
                                                   const Scal* __restrict__ sc, double* __restrict__ part)
{
    constexpr bool STAGE = sizeof(T) == 4;  // FP32 fields fit LDS next to the state
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tu = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[4];
    __shared__ double tinv_s[256];
    __shared__ int s_off[kMaxOffs], s_q[kMaxOffs];
    __shared__ double s_fw[kMaxOffs];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        if (sc && sc[item.x].done) {
            if (threadIdx.x == 0 && part) part[it] = 0.0;
            continue;
        }
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        int halo[3] = {I.dim >= 3 ? I.J : 0, I.dim >= 2 ? I.J : 0, I.J};
        int L[3] = {I.E[0] + 2 * halo[0], I.E[1] + 2 * halo[1], I.E[2] + 2 * halo[2]};
        const int tot = stage_box_len(L);
        T* td = tu + tot;
        T* tc = td + tot;
        const T* p = pvec + I.off;
        const T* dlt = static_cast<const T*>(I.delta);
        const T* cf = static_cast<const T*>(I.coef);
        __syncthreads();
        for (int k = threadIdx.x; k <= I.kmax && k < 256; k += blockDim.x) tinv_s[k] = Tinv[k];
        // this tile's flat LDS offsets of the ball (uniform reads in the pair loop)
        const int nq = I.nq < kMaxOffs ? I.nq : kMaxOffs;
        for (int q = threadIdx.x; q < nq; q += blockDim.x) {
            int4 o = full[q];
            s_off[q] = (o.x * L[1] + o.y) * L[2] + o.z;
            s_q[q] = o.w;
            s_fw[q] = fw[q];
        }
        struct Slot {
            T u, d, c;
        };
        stage_batched(
            tot,
            [&](int idx) {
                int l2 = idx % L[2];
                int r = idx / L[2];
                int l1 = r % L[1];
                int l0 = r / L[1];
                int g0 = org[0] - halo[0] + l0, g1 = org[1] - halo[1] + l1, g2 = org[2] - halo[2] + l2;
                bool in = g0 >= 0 && g0 < ext[0] && g1 >= 0 && g1 < ext[1] && g2 >= 0 && g2 < ext[2];
                int64_t gg = ((int64_t)g0 * ext[1] + g1) * ext[2] + g2;
                Slot v{T(0), T(-1), T(0)};
                if (in) {
                    if (!DIAG) v.u = p[gg];
                    if (STAGE) {
                        v.d = dlt[gg];
                        v.c = cf[gg];
                    }
                }
                return v;
            },
            [&](int idx, const Slot& v) {
                if (!DIAG) tu[idx] = v.u;
                if (STAGE) {
                    td[idx] = v.d;
                    tc[idx] = v.c;
                }
            });
        __syncthreads();
        double dot = 0.0;
        const double nh = 0.5 * (double)I.n;
        const double ch = 0.5 * I.n2;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int r = pi / I.E[2];
            int e1 = r % I.E[1];
            int e0 = r / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            int cidx = ((e0 + halo[0]) * L[1] + (e1 + halo[1])) * L[2] + (e2 + halo[2]);
            double di = STAGE ? (double)td[cidx] : (double)dlt[gi];
            double ci = STAGE ? (double)tc[cidx] : (double)cf[gi];
            double cpi = ci * ch;
            T u0 = DIAG ? T(0) : tu[cidx];
            Acc<T> acc;
            double dsum = 0.0;
            for (int q = 0; q < nq; q++) {
                const int off = s_off[q];
                const int qw = s_q[q];
                double dj, cj;
                if (STAGE) {
                    dj = (double)td[cidx + off];
                    cj = (double)tc[cidx + off];
                    if (dj < 0.0) { dj = di; cj = ci; }
                } else {
                    int4 o = full[q];
                    int y0 = x0 + o.x, y1 = x1 + o.y, y2 = x2 + o.z;
                    dj = di;
                    cj = ci;
                    if (y0 >= 0 && y0 < ext[0] && y1 >= 0 && y1 < ext[1] && y2 >= 0 && y2 < ext[2]) {
                        int64_t gj = ((int64_t)y0 * ext[1] + y1) * ext[2] + y2;
                        dj = (double)dlt[gj];
                        cj = (double)cf[gj];
                    }
                }
                double am = (di + dj) * nh;
                double tt = am * am;
                int kij = (int)ceil(tt) - 1;
                if (qw > kij) continue;
                double w;
                if (DISC) {
                    w = (cpi + cj * ch) * s_fw[q] * (kij < 256 ? tinv_s[kij] : Tinv[kij]);
                } else {
                    double C = 0.5 * (ci + cj);
                    double dij = (di + dj) * 0.5;
                    double dd2 = pow(dij, (double)(I.dim + 2));
                    double base = C * pow(am, -I.expo) * I.hd / dd2 * s_fw[q];
                    w = I.norm == NDL_NORM_CONTINUOUS ? base * I.m2 / I.contc : base;
                }
                if (DIAG) {
                    dsum += w;
                } else {
                    acc.fma_((T)w, tu[cidx + off] - u0);
                    if ((q & 7) == 7) acc.flush();
                }
            }
            T* qv = qvec + I.off;
            if (DIAG) {
                qv[gi] = (T)dsum;
            } else {
                T val = -acc.value();  // A = -L
                qv[gi] = val;
                dot += (double)u0 * (double)val;
            }
        }
        if (part) {
            double s = block_sum(dot, red);
            if (threadIdx.x == 0) part[it] = s;
        }
    }
}

// The same operator for batches of 2D and 3D problems with the discrete
// normalisation, mapped for gfx950: a block covers a 16 x 64 tile (2D, 4
// waves of 4 rows) or an 8 x 4 x 64 tile (3D, 16 waves of 4 rows x 32
// columns), and each lane 4 (2D) or 2 (3D) nodes of one column along
// axis dim-2, so the uniform per-offset work (offset, |z|^2, |z|^e) is shared
// by those nodes and the partner reads of one offset use immediate LDS
// offsets from one address.  A 3D wave ends its offset loop at the bound of
// its own block and the reach around it, which the compact block keeps close
// to its nodes' horizons.
// 2D tiles stage m = delta n/2 in FP64 (exact for FP32 delta, so that
// m_i + m_j is exactly the (delta_i + delta_j) n/2 of the cutoff rule; FP64
// data stage delta and form (delta_i + delta_j) n/2 as the rule writes it);
// 3D tiles (FP32 only) stage delta itself, 4 bytes, and form the same exact
// FP64 value from it, so that the larger haloed tile keeps two waves per
// SIMD.  c n^2/2 and u are staged in the element type.  Per pair:
//   t = a^2 in FP64 with a as above; the pair is in the ball iff |z|^2 < t,
//   i.e. |z|^2 <= ceil(t) - 1 = k_ij;  w = (c'_i + c'_j) |z|^e M / T_e[k_ij]
//   (where the kernel holds the shell-weight table, one lookup of it at
//   (|z|^2, k_ij) gives |z|^e M / T_e[k_ij], or 0 outside the ball).
// The membership test is skipped for offsets inside every pair's ball of the
// tile (|z|^2 < (2 min m)^2) and the loop ends past the largest
// (|z|^2 >= (2 max m)^2); a partner outside Omega takes (delta_i, c_i), which
// only waves with nodes within J of the boundary test for.
// 3D: 2 nodes per lane, 16 waves per 8 x 4 x 64 tile (the haloed tile leaves
// room for one block per CU, so the occupancy comes from the block's waves)
// Tile of one block: 16 x 64 (2D) or 8 x 4 x 64 (3D) nodes, PY nodes per
// lane.  FP64 vectors on 3D problems with FP32 fields (the outer residual of
// the mixed-precision solve) stage 4 planes at a time, in two halves, so that
// the 8-byte u and c' fit the LDS next to the 4-byte horizon.
// Launch variants (the autotuner's search space): nodes per lane PY, which
// sets the block size for the fixed tile, times the persistent grid size.
// Every variant sums each node's pairs in the same order, so all give bitwise
// the same q = -L p; only the block's reduction of the p.q partial differs.
constexpr int kDivPY2[3] = {4, 2, 8};  // 2D, first = default
constexpr int kDivPY3[2] = {2, 4};     // 3D, first = default
constexpr int kDivGrid[3] = {2048, 1024, 4096};
inline int div_num_variants(int dim) { return (dim == 3 ? 2 : 3) * 3; }

template <typename T, int DIM, int PYV>
struct DivShape {
    static constexpr int PY = PYV;
    static constexpr int TY = DIM == 3 ? 4 : 16;
    static constexpr int TZ = DIM == 3 ? (sizeof(T) == 8 ? 4 : 8) : 1;
    static constexpr int SUB = DIM == 3 ? 8 / TZ : 1;  // staged slabs per item
    static constexpr int THREADS = 64 * TZ * TY / PY;
};

// offs: per ball offset, sorted by |z|^2, {the partner's offset in the staged
// tile, |z|^2, the start of the shell's weight row less one, 0}, then a
// sentinel (built with the batch's tables on the host).
template <typename T, typename D, bool DIAG, int JT, int DIM, int PYV>
__global__ __launch_bounds__((DivShape<T, DIM, PYV>::THREADS)) void k_div2_items(
    const Inst* __restrict__ insts, const int2* __restrict__ items, int nitems, const T* __restrict__ pvec,
    T* __restrict__ qvec, const int4* __restrict__ offs, const double* __restrict__ fw, const double* __restrict__ Tinv,
    const Scal* __restrict__ sc, double* __restrict__ part)
{
    using SH = DivShape<T, DIM, PYV>;
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int PY = SH::PY;
    constexpr int NWAVES = SH::THREADS / 64;
    // staged horizon: MT values; SC = already scaled by n/2 (2D FP32 only)
    using MT = typename std::conditional<DIM == 3, float, double>::type;
    constexpr bool SC = DIM == 2 && F32;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2 * NWAVES];
    __shared__ T tinv_s[256];
    __shared__ int s_q[kMaxOffs];
    __shared__ T s_fw[kMaxOffs];  // profile weight |z|^expo of the offsets, in the vectors' type
    // shell-weight table: 3D, and 2D FP32 vectors up to reach 7 (a larger
    // table would cost the 2D tile a block per unit)
    constexpr int KW = w2_width(DIM, JT);
    constexpr bool TABOK = DIM == 3 || (sizeof(T) == 4 && JT <= 7);
    __shared__ T s_w2[TABOK ? KW * KW : 1];
    // 3D: per staged plane and column, the largest staged delta over the
    // tile's rows (each wave's loop bound is read from it)
    static_assert(DIM != 3 || (SH::TY == 4 && PYV >= 2), "3D waves cover the tile's 4 rows");
    constexpr int kCM = DIM == 3 ? (SH::TZ + 2 * JT) * (64 + 2 * JT) : 1;
    __shared__ float s_cmax[kCM];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        const Inst I = insts[item.x];
        if (sc && sc[item.x].done) {
            if (threadIdx.x == 0 && part) part[it] = 0.0;
            continue;
        }
        int org[3];
        item_geom<T>(I, item.y, org);
        double dot = 0.0;
        for (int sub = 0; sub < SH::SUB; ++sub) {
        // every problem of the batch uses the halo JT >= its own J, so the tile
        // pitch is a compile-time constant and the partner reads of the PY
        // nodes of a lane use immediate offsets
        const int n = I.n;
        constexpr int J = JT;
        constexpr int TZ = SH::TZ, TY = SH::TY, HZ = DIM == 3 ? J : 0;
        constexpr int PITCH = 64 + 2 * J, SY = TY + 2 * J, SZ = TZ + 2 * HZ;
        constexpr int PLANE = SY * PITCH, tot = SZ * PLANE;
        // LDS tile: horizon m, coefficient c and vector u of every staged node.
        // In 3D, FP32 vectors keep a node's three values side by side (one
        // address per offset for the reads of both nodes of a lane); FP64
        // vectors keep three arrays (side by side they would not fit the 3D
        // tile), and so does 2D (its rows of 4 nodes per lane reach past the
        // paired-read offset range either way)
        constexpr bool AOS = F32 && DIM == 3;
        struct Node {
            MT m;
            T c, u;
        };
        static_assert(!AOS || sizeof(Node) == sizeof(MT) + 2 * sizeof(T), "packed node");
        Node* tn = reinterpret_cast<Node*>(smem_raw);
        MT* tm = reinterpret_cast<MT*>(smem_raw);
        T* tcc = reinterpret_cast<T*>(tm + tot);
        T* tu = tcc + tot;
        auto lm = [&](int i) -> MT& {
            if constexpr (AOS) return tn[i].m;
            else return tm[i];
        };
        auto lc = [&](int i) -> T& {
            if constexpr (AOS) return tn[i].c;
            else return tcc[i];
        };
        auto lu = [&](int i) -> T& {
            if constexpr (AOS) return tn[i].u;
            else return tu[i];
        };
        const T* p = pvec + I.off;
        const D* dlt = static_cast<const D*>(I.delta);
        const D* cf = static_cast<const D*>(I.coef);
        const double nh = 0.5 * (double)n;
        const double ch = 0.5 * I.n2;
        __syncthreads();  // the previous item's readers are done
        for (int k = threadIdx.x; k <= I.kmax && k < 256; k += blockDim.x) tinv_s[k] = (T)Tinv[k];
        const bool tab = TABOK && I.wtab;
        if (tab)
            for (int e = threadIdx.x; e < KW * KW; e += blockDim.x) s_w2[e] = (T)Tinv[kW2Off + e];
        const int nq = I.nq < kMaxOffs ? I.nq : kMaxOffs;
        for (int q = threadIdx.x; q < nq; q += blockDim.x) {
            s_q[q] = offs[q].y;
            s_fw[q] = (T)fw[q];
        }
        const int z0 = org[0] + sub * TZ, y0 = org[1], x0 = org[2];
        const int nz = DIM == 3 ? n : 1;
        double mmax = 0.0, mmin = 1e300;
        struct Slot {
            D d, c;
            T u;
            bool in;
        };
        stage_batched(
            tot,
            [&](int idx) {
                const int sz = idx / PLANE, rem = idx - sz * PLANE;
                const int r = rem / PITCH, c = rem - r * PITCH;
                const int gz = z0 - HZ + sz, gy = y0 - J + r, gx = x0 - J + c;
                const bool in = gz >= 0 && gz < nz && gy >= 0 && gy < n && gx >= 0 && gx < n;
                const int64_t gg = ((int64_t)gz * n + gy) * n + gx;
                Slot v{D(0), D(0), T(0), in};
                if (in) {
                    v.d = dlt[gg];
                    v.c = cf[gg];
                    if (!DIAG) v.u = p[gg];
                }
                return v;
            },
            [&](int idx, const Slot& v) {
                MT m = MT(-1);
                T cc = 0;
                if (v.in) {
                    m = SC ? (MT)((double)v.d * nh) : (MT)v.d;
                    cc = (T)((double)v.c * ch);
                    const double ms = SC ? (double)m : (double)m * nh;
                    mmax = fmax(mmax, ms);
                    mmin = fmin(mmin, ms);
                }
                lm(idx) = m;
                lc(idx) = cc;
                lu(idx) = v.u;
            });
        if constexpr (DIM == 3) {
            __syncthreads();  // the staged tile is complete
            for (int e = threadIdx.x; e < SZ * PITCH; e += blockDim.x) {
                const int sz = e / PITCH, c = e - sz * PITCH;
                float v = 0.f;  // nodes outside Omega hold -1
#pragma unroll
                for (int r = 0; r < SY; ++r) v = fmaxf(v, (float)lm(sz * PLANE + r * PITCH + c));
                s_cmax[e] = v;
            }
        }
        // block extremes of m (uniform loop bounds)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mmax = fmax(mmax, __shfl_xor(mmax, o, 64));
            mmin = fmin(mmin, __shfl_xor(mmin, o, 64));
        }
        if (lane == 0) {
            red[wv] = mmax;
            red[NWAVES + wv] = mmin;
        }
        __syncthreads();
        mmax = red[0];
        mmin = red[NWAVES];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) {
            mmax = fmax(mmax, red[w]);
            mmin = fmin(mmin, red[NWAVES + w]);
        }
        const double tmax = 4.0 * mmax * mmax;  // (2 max m)^2 >= every t of the tile
        const double tmin = 4.0 * mmin * mmin;

        // the lane's nodes: column wx, rows wy .. wy + PY - 1 of plane wz.
        // 2D: wave wv holds rows PY wv .. PY wv + PY - 1, one node column per
        // lane.  3D: wave wv holds a 32-column x 4-row x PY/2-plane block
        // (column half xh, plane group zg), each half-wave 32 consecutive
        // columns (consecutive nodes of the staged tile), so that its nodes'
        // horizons, and with them its offset loop, span less than a full
        // tile row would (the horizon varies along the rows).  Waves wv and
        // wv + 4 share a SIMD and take opposite halves, which balances the
        // SIMDs' loops.
        constexpr int ZL = DIM == 3 ? PY / 2 : 1;  // planes per wave
        const int xh = NWAVES >= 8 ? (wv >> 2) & 1 : wv & 1;
        const int zg = NWAVES >= 8 ? (wv & 3) + 4 * (wv >> 3) : wv >> 1;
        int wx, wy, wz;
        if constexpr (DIM == 3) {
            constexpr int YG = SH::TY / PY;  // row groups of a wave (2 or 1)
            const int h = lane >> 5;
            wx = xh * 32 + (lane & 31);
            wy = (h % YG) * PY;
            wz = zg * ZL + h / YG;
        } else {
            constexpr int WPP = SH::TY / PY;  // waves per plane
            wx = lane;
            wy = (wv % WPP) * PY;
            wz = wv / WPP;
        }
        const int x = x0 + wx;
        const int base = (wz + HZ) * PLANE + (wy + J) * PITCH + wx + J;
        // a partner of one of the wave's nodes lies outside Omega (or the wave
        // holds nodes past the grid): the wave takes the pair loop that
        // substitutes the node's own horizon and coefficient for such partners
        bool edge;
        if constexpr (DIM == 3) {
            const int zb = z0 + zg * ZL, xb = x0 + xh * 32;
            edge = zb - HZ < 0 || zb + ZL + HZ > nz || y0 - J < 0 || y0 + TY + J > n || xb - J < 0 ||
                   xb + 32 + J > n;
        } else {
            const int yb = y0 + wy;  // the wave's first row
            edge = yb - J < 0 || yb + PY + J > n || x0 - J < 0 || x0 + 64 + J > n;
        }
        double mi[PY], mh[PY];  // m of the node (scaled by n/2 when SC), and m n / 2
        T cci[PY], ui[PY];
        bool valid[PY];
        Acc<T> acc[PY];
        double dsum[PY];
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            // nodes past the grid edge (ragged tiles) compute with c = 0 and the
            // tile's largest horizon, so that every pair they form has m_ij > 0
            // and 0 <= k_ij <= k_max (within the table); they are not stored
            valid[j] = x < n && y0 + wy + j < n && z0 + wz < nz;
            mi[j] = valid[j] ? (double)lm(base + j * PITCH) : (SC ? mmax : mmax / nh);
            // m n / 2 is exact in FP64 (an FP32 m times n / 2), so that
            // fma(m_j, n / 2, m_i n / 2) rounds (m_i + m_j) n / 2 once, as the
            // product of the exact sum does
            mh[j] = SC ? mi[j] : (valid[j] ? mi[j] * nh : mmax);
            cci[j] = valid[j] ? lc(base + j * PITCH) : T(0);
            ui[j] = lu(base + j * PITCH);
            dsum[j] = 0.0;
        }
        // offsets [0, p_in) lie inside every pair's ball of the tile, [p_in, p_end)
        // need the per-pair test, the rest lie outside every ball (the table
        // is sorted by |z|^2; uniform binary searches)
        auto first_at_least = [&](double tq) {
            int lo = 0, hi = nq;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((double)s_q[mid] < tq) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        double tend = tmax;
        if constexpr (DIM == 3) {
            // a 3D wave's pairs join nodes of its planes and columns widened by
            // the reach J (all rows of the tile): (2 max m)^2 over that region
            // bounds their t, computed as the tile's bound is
            const int zb = zg * ZL, xb = xh * 32;
            constexpr int RW = 32 + 2 * J;  // region columns, one per lane
            static_assert(RW <= 64, "one region column per lane");
            float wm = 0.f;
            if (lane < RW) {
#pragma unroll
                for (int pz = 0; pz < ZL + 2 * HZ; ++pz) wm = fmaxf(wm, s_cmax[(zb + pz) * PITCH + xb + lane]);
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) wm = fmaxf(wm, __shfl_xor(wm, o, 64));
            wm = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wm)));
            const double ws = (double)wm * nh;
            tend = fmin(tmax, 4.0 * ws * ws);
        }
        const int p_end = first_at_least(tend);
        const int p_in = min(first_at_least(tmin), p_end);
        // per-lane bases of the staged fields: a partner read is the base plus
        // the uniform offset (one add per offset for the interleaved tile, one
        // per field for the three arrays)
        // the interleaved tile's lane base as an LDS pointer the compiler
        // cannot split (its constant part would otherwise be re-added per
        // offset to reach the paired-read offset range)
        using LdsNode = const Node __attribute__((address_space(3)));
        LdsNode* tnb = (LdsNode*)(tn + base);
        asm volatile("" : "+v"(tnb));
        const MT* tmb = tm + base;
        const T* tcb = tcc + base;
        const T* tub = tu + base;
        // one range of offsets; the table entries are uniform (scalar loads)
        auto run = [&](int pb, int pe, auto edge_c, auto mask_c, auto tab_c) {
            constexpr bool EDGE = decltype(edge_c)::value;
            constexpr bool MASK = decltype(mask_c)::value;
            constexpr bool TAB = decltype(tab_c)::value;
            if (pb >= pe) return;
            // the table entries of the next offset are loaded one iteration
            // ahead (the table carries one sentinel entry past its end)
            int4 o = offs[pb];
            for (int q = pb; q < pe; ++q) {
                const int off = o.x;  // the partner's offset in the staged tile
                const int qi = o.y;   // |z|^2 >= 1: the table holds no zero offset
                const T fq = TAB ? T(0) : s_fw[q];
                // the row of the shell, shifted by one so that it is indexed
                // by ceil(t) = k_ij + 1 (one address add per pair)
                const T* wrow = s_w2 + (TAB ? o.z : 0);
                o = offs[q + 1];
#pragma unroll
                for (int j = 0; j < PY; ++j) {
                    const int jo = j * PITCH + off;
                    LdsNode* np = tnb + off;
                    double mj = AOS ? (double)np[j * PITCH].m : (double)tmb[jo];
                    T ccj = AOS ? np[j * PITCH].c : tcb[jo];
                    if (EDGE) {
                        const bool out = mj < 0.0;
                        mj = out ? mi[j] : mj;
                        ccj = out ? cci[j] : ccj;
                    }
                    const double a = SC ? mi[j] + mj : fma(mj, nh, mh[j]);
                    const double t = a * a;
                    const int ct = (int)ceil(t);
                    const int kij = ct - 1;
                    // |z|^2 < t  <=>  |z|^2 <= ceil(t) - 1 = k_ij for an integer |z|^2
                    T w;
                    if (TAB) {
                        w = (cci[j] + ccj) * wrow[ct];  // zero outside the ball
                    } else {
                        const bool inside = qi <= kij;
                        w = (cci[j] + ccj) * tinv_s[kij] * fq;
                        if (MASK) w = inside ? w : T(0);
                    }
                    if (DIAG) {
                        dsum[j] += (double)w;
                    } else {
                        acc[j].fma_(w, (AOS ? np[j * PITCH].u : tub[jo]) - ui[j]);
                    }
                }
                if (!DIAG && F32 && (q & 7) == 7) {
#pragma unroll
                    for (int j = 0; j < PY; ++j) acc[j].flush();
                }
            }
        };
        using yes = std::integral_constant<bool, true>;
        using no = std::integral_constant<bool, false>;
        if (tab) {
            if (edge) {
                run(0, p_in, yes{}, no{}, yes{});
                run(p_in, p_end, yes{}, yes{}, yes{});
            } else {
                run(0, p_in, no{}, no{}, yes{});
                run(p_in, p_end, no{}, yes{}, yes{});
            }
        } else if (edge) {
            run(0, p_in, yes{}, no{}, no{});
            run(p_in, p_end, yes{}, yes{}, no{});
        } else {
            run(0, p_in, no{}, no{}, no{});
            run(p_in, p_end, no{}, yes{}, no{});
        }
        T* qv = qvec + I.off;
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            if (!valid[j]) continue;
            const int64_t gi = ((int64_t)(z0 + wz) * n + (y0 + wy + j)) * n + x;
            if (DIAG) {
                qv[gi] = (T)dsum[j];
            } else {
                const T val = -acc[j].value();  // A = -L
                qv[gi] = val;
                dot += (double)ui[j] * (double)val;
            }
        }
        }  // slabs of the item
        if (part) {
            const double s = block_sum(dot, red);
            if (threadIdx.x == 0) part[it] = s;
        }
    }
}

// x += alpha p; r -= alpha q; z = r / diag; partials of r.z and r.r
template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                   int nitems, const Scal* __restrict__ sc, T* __restrict__ x,
                                                   T* __restrict__ r, T* __restrict__ z, const T* __restrict__ p,
                                                   const T* __restrict__ q, const T* __restrict__ dinv,
                                                   double* __restrict__ part_rz, double* __restrict__ part_rr)
{
    __shared__ double red[4];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        const Scal S = sc[item.x];
        if (S.done) {
            if (threadIdx.x == 0) { part_rz[it] = 0.0; part_rr[it] = 0.0; }
            continue;
        }
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        T a = (T)S.alpha;
        double drz = 0.0, drr = 0.0;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            x[gi] += a * p[gi];
            T rv = r[gi] - a * q[gi];
            r[gi] = rv;
            T zv = rv * dinv[gi];
            z[gi] = zv;
            drz += (double)rv * (double)zv;
            drr += (double)rv * (double)rv;
        }
        double s1 = block_sum(drz, red);
        double s2 = block_sum(drr, red);
        if (threadIdx.x == 0) { part_rz[it] = s1; part_rr[it] = s2; }
    }
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void k_cg_dir(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                int nitems, const Scal* __restrict__ sc, const T* __restrict__ z,
                                                T* __restrict__ p)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        if (sc[item.x].done) continue;
        T b = (T)sc[item.x].beta;
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            p[gi] = z[gi] + b * p[gi];
        }
    }
}

// Sum of a problem's item partials by one block (fixed order: strided
// per-thread sums, then a tree), valid in thread 0.
__device__ __forceinline__ double problem_sum(const Inst& I, const double* __restrict__ part, double* sh)
{
    double a = 0.0;
    for (int t = threadIdx.x; t < I.nitems; t += blockDim.x) a += part[I.item0 + t];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Per-problem scalar steps (one thread per problem, items summed in order).
// phase 0: alpha = rz / p.q ; phase 1: rz_new, rr -> beta, convergence flag.
__global__ void k_cg_scalars(int nprob, const Inst* __restrict__ insts, Scal* __restrict__ sc,
                             const double* __restrict__ p0, const double* __restrict__ p1, int phase, int max_iter)
{
    __shared__ double sh[256];
    int i = blockIdx.x;
    if (i >= nprob) return;
    if (sc[i].done) return;
    const Inst I = insts[i];
    double s0 = problem_sum(I, p0, sh);
    double s1 = phase == 1 ? problem_sum(I, p1, sh) : 0.0;
    if (threadIdx.x != 0) return;
    Scal S = sc[i];
    if (phase == 0) {
        double pq = s0;
        S.pq = pq;
        S.alpha = (pq > 0.0 && isfinite(pq)) ? S.rz / pq : 0.0;
        if (!(pq > 0.0) || !isfinite(pq)) S.done = 3;  // breakdown: not SPD or NaN
    } else {
        double rz = s0, rr = s1;
        S.rz_new = rz;
        S.rr = rr;
        S.beta = S.rz != 0.0 ? rz / S.rz : 0.0;
        S.rz = rz;
        S.iters += 1;
        if (rr <= S.tol2) S.done = 1;
        else if (S.iters >= max_iter) S.done = 2;
        else if (!isfinite(rr)) S.done = 3;
    }
    sc[i] = S;
}

// Initialisation of an inner solve: p = z = r / diag; partial r.z, r.r.
template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                 int nitems, T* __restrict__ x, const T* __restrict__ r,
                                                 T* __restrict__ z, T* __restrict__ p, const T* __restrict__ dinv,
                                                 double* __restrict__ part_rz, double* __restrict__ part_rr)
{
    __shared__ double red[4];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        double drz = 0.0, drr = 0.0;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            T rv = r[gi];
            T zv = rv * dinv[gi];
            z[gi] = zv;
            p[gi] = zv;
            x[gi] = T(0);
            drz += (double)rv * (double)zv;
            drr += (double)rv * (double)rv;
        }
        double s1 = block_sum(drz, red);
        double s2 = block_sum(drr, red);
        if (threadIdx.x == 0) { part_rz[it] = s1; part_rr[it] = s2; }
    }
}

__global__ void k_cg_start(int nprob, const Inst* __restrict__ insts, Scal* __restrict__ sc,
                           const double* __restrict__ prz, const double* __restrict__ prr, const double* __restrict__ tol2)
{
    __shared__ double sh[256];
    int i = blockIdx.x;
    if (i >= nprob) return;
    const Inst I = insts[i];
    double rz = problem_sum(I, prz, sh);
    double rr = problem_sum(I, prr, sh);
    if (threadIdx.x != 0) return;
    Scal S = sc[i];
    S.rz = rz;
    S.rr = rr;
    S.tol2 = tol2[i];
    S.alpha = S.beta = 0.0;
    S.done = (rr <= S.tol2) ? 1 : 0;
    sc[i] = S;
}

// ------------------------------------------------------------------ FP64 outer helpers
// r = b - A x (A = -L, x FP64), partial ||r||^2 per item; rin = r * scale (inner type)
template <typename T>
__global__ __launch_bounds__(256) void k_residual(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                  int nitems, const double* __restrict__ b,
                                                  const double* __restrict__ ax, double* __restrict__ r,
                                                  double* __restrict__ part)
{
    __shared__ double red[4];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        double acc = 0.0;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            double v = b[gi] - ax[gi];
            r[gi] = v;
            acc += v * v;
        }
        double s = block_sum(acc, red);
        if (threadIdx.x == 0) part[it] = s;
    }
}

// one block per problem
__global__ void k_item_sums(int nprob, const Inst* __restrict__ insts, const double* __restrict__ part,
                            double* __restrict__ out)
{
    __shared__ double sh[256];
    int i = blockIdx.x;
    if (i >= nprob) return;
    const Inst I = insts[i];
    double s = problem_sum(I, part, sh);
    if (threadIdx.x == 0) out[i] = s;
}

// elementwise over the concatenated vectors: dst = (To)(src * scale[prob])
template <typename To, typename Ti>
__global__ void k_scale_copy(const Inst* __restrict__ insts, const int* __restrict__ owner, int64_t total,
                             const Ti* __restrict__ src, To* __restrict__ dst, const double* __restrict__ scale)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int pr = owner[i >> 10];
    double sc = scale ? scale[pr] : 1.0;
    dst[i] = (To)((double)src[i] * sc);
}

// x64 += d / scale[prob]  (scale = 1 / ||r|| of the inner right-hand side)
template <typename T>
__global__ void k_axpy_outer(const int* __restrict__ owner, int64_t total, double* __restrict__ x,
                             const T* __restrict__ d, const double* __restrict__ scale, const int* __restrict__ active)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int pr = owner[i >> 10];
    if (!active[pr]) return;
    x[i] += (double)d[i] / scale[pr];
}

template <typename T>
__global__ void k_recip(const T* __restrict__ dg, T* __restrict__ dv, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dv[i] = dg[i] != T(0) ? T(1) / dg[i] : T(0);
}

__global__ void k_fill_f64(double* p, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ host driver
struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

template <typename T>
static int alloc(DevBuf& b, size_t count)
{
    NDL_HIP(hipMalloc(&b.p, std::max<size_t>(count, 1) * sizeof(T)));
    return NDL_OK;
}

static double sphere_area_s(int d) { return d == 1 ? 2.0 : (d == 2 ? 2.0 * M_PI : 4.0 * M_PI); }

static double radial_moment_s(const Plan& p)
{
    int d = p.dim;
    switch (p.kernel) {
    case NDL_G_CONST: return 1.0 / (d + 2.0);
    case NDL_G_INV_R: return 1.0 / (d + 1.0);
    default: return 1.0 / (2.0 - 2.0 * p.prob.s);
    }
}

struct Batch {
    std::vector<Inst> insts;
    std::vector<int2> items;
    std::vector<int> owner;  // problem of each 1024-element chunk of the concatenated vectors
    int64_t total = 0;
    int dim = 0, Jmax = 0;
    int64_t kmax = 0;
    int variant = 0;         // launch variant of the specialised item kernel (autotuned)
};

static int build_batch(const ndl_plan* plans, int nprob, Batch& B, bool f64_fields, std::vector<DevBuf>& keep)
{
    for (int i = 0; i < nprob; ++i) {
        const Plan& p = *reinterpret_cast<const Plan*>(plans[i]);
        if ((int)ball_offsets(p.dim, p.kmax, false).size() > kMaxOffs) {
            set_error("solver: horizon ball of problem %d has more than %d offsets", i, kMaxOffs);
            return NDL_EUNSUPPORTED;
        }
    }
    B.insts.resize(nprob);
    int64_t off = 0;
    for (int i = 0; i < nprob; ++i) {
        const Plan& p = *reinterpret_cast<const Plan*>(plans[i]);
        Inst I{};
        I.dim = p.dim;
        I.n = (int)p.n;
        I.J = p.J;
        I.kmax = (int)p.kmax;
        I.nq = (int)ball_offsets(p.dim, p.kmax, false).size();
        if (p.dim == 2) { I.E[0] = 1; I.E[1] = 16; I.E[2] = 64; }
        else if (p.dim == 3) { I.E[0] = 8; I.E[1] = 4; I.E[2] = 64; }
        else { I.E[0] = 1; I.E[1] = 1; I.E[2] = 1024; }
        int ext[3] = {p.dim >= 3 ? (int)p.n : 1, p.dim >= 2 ? (int)p.n : 1, (int)p.n};
        int nt = 1;
        for (int a = 0; a < 3; ++a) {
            I.tiles[a] = (ext[a] + I.E[a] - 1) / I.E[a];
            nt *= I.tiles[a];
        }
        I.N = p.N;
        I.off = off;
        off += ((p.N + 1023) / 1024) * 1024;  // chunk-aligned so each 1024-chunk has one owner
        I.item0 = (int)B.items.size();
        I.nitems = nt;
        for (int t = 0; t < nt; ++t) B.items.push_back(make_int2(i, t));
        I.delta = p.prob.delta;
        I.coef = p.prob.coef;
        I.n2 = (double)p.n * (double)p.n;
        I.norm = p.norm;
        I.expo = p.expo;
        I.m2 = p.m2;
        I.contc = sphere_area_s(p.dim) * radial_moment_s(p);
        double hd = 1.0;
        for (int a = 0; a < p.dim; ++a) hd /= (double)p.n;
        I.hd = hd;
        B.insts[i] = I;
        B.Jmax = std::max(B.Jmax, p.J);
        B.kmax = std::max<int64_t>(B.kmax, p.kmax);
        B.dim = p.dim;
    }
    B.total = off;
    for (auto& I : B.insts) I.wtab = B.kmax < w2_width(B.dim, B.Jmax) ? 1 : 0;
    B.owner.assign(off / 1024, 0);
    for (int i = 0; i < nprob; ++i)
        for (int64_t c = B.insts[i].off / 1024; c < (B.insts[i].off + B.insts[i].N + 1023) / 1024; ++c) B.owner[c] = i;
    (void)f64_fields;
    (void)keep;
    return NDL_OK;
}

template <typename T>
static __global__ void k_widen(const T* __restrict__ a, double* __restrict__ b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Batches with the discrete normalisation run the specialised kernel: 2D with
// halo J <= 8, and 3D with J <= 3 for FP32 vectors, or FP64 vectors over FP32
// fields (f32data: the outer residual of the mixed-precision solve); the
// haloed tile must fit the LDS of one CU.
template <typename T>
static bool use_div_spec(const Batch& B, bool f32data = false)
{
    if (B.insts[0].norm != NDL_NORM_DISCRETE || B.kmax >= 256 || B.Jmax < 1) return false;
    if (B.dim == 2) return B.Jmax <= 8;
    if (B.dim == 3) return (sizeof(T) == 4 || f32data) && B.Jmax <= 3;
    return false;
}

template <typename T>
static size_t items_lds(const Batch& B, bool f32data = false)
{
    const Inst& I0 = B.insts[0];
    if (use_div_spec<T>(B, f32data)) {
        const int J = B.Jmax;
        size_t cells;
        if (B.dim == 3) cells = (size_t)(DivShape<T, 3, 2>::TZ + 2 * J) * (DivShape<T, 3, 2>::TY + 2 * J) * (64 + 2 * J);
        else cells = (size_t)(DivShape<T, 2, 4>::TY + 2 * J) * (64 + 2 * J);
        return cells * ((B.dim == 3 ? sizeof(float) : sizeof(double)) + 2 * sizeof(T));
    }
    int L[3] = {I0.E[0] + (B.dim >= 3 ? 2 * B.Jmax : 0), I0.E[1] + (B.dim >= 2 ? 2 * B.Jmax : 0),
                I0.E[2] + 2 * B.Jmax};
    size_t cells = (size_t)L[0] * L[1] * L[2];
    return cells * sizeof(T) * (sizeof(T) == 4 ? 3 : 1);
}

// every instantiation of the specialised item kernel for element type T and
// field type DT in dim DD (reaches 1..JMAX, all launch variants, DIAG at the
// default variant)
template <typename T, typename DT, int DD, int JJ>
static void div2_kernels_j(std::vector<const void*>& v)
{
    constexpr int P0 = DD == 3 ? kDivPY3[0] : kDivPY2[0];
    v.push_back((const void*)k_div2_items<T, DT, true, JJ, DD, P0>);
    if constexpr (DD == 3) {
        v.push_back((const void*)k_div2_items<T, DT, false, JJ, DD, kDivPY3[0]>);
        v.push_back((const void*)k_div2_items<T, DT, false, JJ, DD, kDivPY3[1]>);
    } else {
        v.push_back((const void*)k_div2_items<T, DT, false, JJ, DD, kDivPY2[0]>);
        v.push_back((const void*)k_div2_items<T, DT, false, JJ, DD, kDivPY2[1]>);
        v.push_back((const void*)k_div2_items<T, DT, false, JJ, DD, kDivPY2[2]>);
    }
}

template <typename T, typename DT, int DD>
static std::vector<const void*> div2_kernels()
{
    std::vector<const void*> v;
    div2_kernels_j<T, DT, DD, 1>(v);
    div2_kernels_j<T, DT, DD, 2>(v);
    div2_kernels_j<T, DT, DD, 3>(v);
    if constexpr (DD == 2) {
        div2_kernels_j<T, DT, DD, 4>(v);
        div2_kernels_j<T, DT, DD, 5>(v);
        div2_kernels_j<T, DT, DD, 6>(v);
        div2_kernels_j<T, DT, DD, 7>(v);
        div2_kernels_j<T, DT, DD, 8>(v);
    }
    return v;
}

template <typename T>
static int prepare_lds(const Batch& B, bool f32data = false)
{
    size_t lds = items_lds<T>(B, f32data);
    if (lds + 16 * 1024 > 160 * 1024) {
        set_error("solver tile needs %zu B of LDS (horizon too wide)", lds);
        return NDL_EUNSUPPORTED;
    }
    // plus ~14 KiB of static LDS (reduction, tables)
    if (lds + 16 * 1024 > 64 * 1024) {
        std::vector<const void*> fns = {(const void*)k_div_items<T, false, true>,
                                        (const void*)k_div_items<T, true, true>,
                                        (const void*)k_div_items<T, false, false>,
                                        (const void*)k_div_items<T, true, false>};
        for (const void* f : div2_kernels<T, T, 2>()) fns.push_back(f);
        for (const void* f : div2_kernels<T, T, 3>()) fns.push_back(f);
        if (f32data && sizeof(T) == 8)
            for (const void* f : div2_kernels<double, float, 3>()) fns.push_back(f);
        for (const void* f : fns) NDL_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    return NDL_OK;
}

template <typename T, typename DT, int JJ, int DD, int PY>
static void launch_div2(unsigned g, size_t lds, hipStream_t s, const Inst* d_insts, const int2* d_items, int nitems,
                        const T* p, T* q, const int4* full, const double* fw, const double* Tinv, const Scal* sc,
                        double* part)
{
    constexpr unsigned nt = (unsigned)DivShape<T, DD, PY>::THREADS;
    k_div2_items<T, DT, false, JJ, DD, PY><<<g, nt, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, Tinv, sc,
                                                              part);
}

template <typename T, typename DT, int JJ, int DD>
static void launch_div2_v(int variant, bool diag, unsigned nitems_u, size_t lds, hipStream_t s,
                          const Inst* d_insts, const int2* d_items, const T* p, T* q, const int4* full,
                          const double* fw, const double* Tinv, const Scal* sc, double* part)
{
    const int nitems = (int)nitems_u;
    const int gi = variant % 3, pi = variant / 3;
    const unsigned g = (unsigned)std::min(nitems, kDivGrid[gi]);
    if (diag) {
        constexpr int P0 = DD == 3 ? kDivPY3[0] : kDivPY2[0];
        constexpr unsigned nt = (unsigned)DivShape<T, DD, P0>::THREADS;
        const unsigned gd = (unsigned)std::min(nitems, kDivGrid[0]);
        k_div2_items<T, DT, true, JJ, DD, P0><<<gd, nt, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, Tinv,
                                                                  sc, part);
        return;
    }
    if constexpr (DD == 3) {
        if (pi == 1) launch_div2<T, DT, JJ, DD, kDivPY3[1]>(g, lds, s, d_insts, d_items, nitems, p, q, full, fw, Tinv, sc, part);
        else launch_div2<T, DT, JJ, DD, kDivPY3[0]>(g, lds, s, d_insts, d_items, nitems, p, q, full, fw, Tinv, sc, part);
    } else {
        if (pi == 1) launch_div2<T, DT, JJ, DD, kDivPY2[1]>(g, lds, s, d_insts, d_items, nitems, p, q, full, fw, Tinv, sc, part);
        else if (pi == 2) launch_div2<T, DT, JJ, DD, kDivPY2[2]>(g, lds, s, d_insts, d_items, nitems, p, q, full, fw, Tinv, sc, part);
        else launch_div2<T, DT, JJ, DD, kDivPY2[0]>(g, lds, s, d_insts, d_items, nitems, p, q, full, fw, Tinv, sc, part);
    }
}

// q = -L p over the items.  f32data: the items' fields are FP32 while the
// vectors are FP64 (3D specialised kernel only; otherwise the caller passes
// FP64 fields).  variant < 0: the batch's tuned variant.
template <typename T>
static int launch_div_items(const Batch& B, const Inst* d_insts, const int2* d_items, const T* p, T* q,
                            const int4* full, const double* fw, int nfull, const double* Tinv, const Scal* sc,
                            double* part, bool diag, hipStream_t s, bool f32data = false, int variant = -1)
{
    size_t lds = items_lds<T>(B, f32data);
    int nitems = (int)B.items.size();
    unsigned g = (unsigned)std::min(nitems, 256 * 8);
    bool disc = B.insts[0].norm == NDL_NORM_DISCRETE;
    if (use_div_spec<T>(B, f32data)) {
        const int v = variant >= 0 ? variant : B.variant;
        const int key = B.dim * 16 + B.Jmax;
#define NDL_DIV2_CASE(DD, JJ, DT)                                                                                 \
    case DD * 16 + JJ:                                                                                            \
        launch_div2_v<T, DT, JJ, DD>(v, diag, (unsigned)nitems, lds, s, d_insts, d_items, p, q, full + nfull, fw, \
                                     Tinv, sc, part);                                                             \
        break;
        if (f32data && sizeof(T) == 8) {
            if constexpr (sizeof(T) == 8) {
                switch (key) {
                    NDL_DIV2_CASE(3, 1, float)
                    NDL_DIV2_CASE(3, 2, float)
                    NDL_DIV2_CASE(3, 3, float)
                default: return NDL_EUNSUPPORTED;
                }
            }
        } else {
            switch (key) {
                NDL_DIV2_CASE(2, 1, T)
                NDL_DIV2_CASE(2, 2, T)
                NDL_DIV2_CASE(2, 3, T)
                NDL_DIV2_CASE(2, 4, T)
                NDL_DIV2_CASE(2, 5, T)
                NDL_DIV2_CASE(2, 6, T)
                NDL_DIV2_CASE(2, 7, T)
                NDL_DIV2_CASE(2, 8, T)
                NDL_DIV2_CASE(3, 1, T)
                NDL_DIV2_CASE(3, 2, T)
                NDL_DIV2_CASE(3, 3, T)
            default: return NDL_EUNSUPPORTED;
            }
        }
#undef NDL_DIV2_CASE
        NDL_HIP(hipGetLastError());
        return NDL_OK;
    }
    if (f32data) {
        set_error("internal: FP32 fields with FP64 vectors need the specialised kernel");
        return NDL_EINVAL;
    }
    if (diag && disc)
        k_div_items<T, true, true><<<g, 256, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, nfull, Tinv, sc, part);
    else if (diag)
        k_div_items<T, true, false><<<g, 256, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, nfull, Tinv, sc, part);
    else if (disc)
        k_div_items<T, false, true><<<g, 256, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, nfull, Tinv, sc, part);
    else
        k_div_items<T, false, false><<<g, 256, lds, s>>>(d_insts, d_items, nitems, p, q, full, fw, nfull, Tinv, sc, part);
    NDL_HIP(hipGetLastError());
    return NDL_OK;
}

// The batch's shared ball tables: the offsets sorted by |z|^2 (plus one
// sentinel entry, as the 2D kernel reads one entry ahead), their profile
// weights |z|^e, and the discrete normalisation M / T_e[k] for k <= kmax
// (T_e[k] = sum over the offsets with |z|^2 <= k of |z|^(e+2)), followed by
// the shell-weight table when kmax < w2_width(dim, J).
static int ball_tables(const Batch& B, double expo, double m2, std::vector<int4>& fb, std::vector<double>& fwv,
                       std::vector<double>& Tinv)
{
    const std::vector<Off> full = ball_offsets(B.dim, B.kmax, false);
    fb.clear();
    fwv.clear();
    for (auto& o : full) {
        fb.push_back(box_offset(B.dim, o));
        fwv.push_back(std::pow(std::sqrt((double)o.q), expo));
    }
    fb.push_back(make_int4(0, 0, 0, 1 << 30));
    fwv.push_back(0.0);
    std::vector<double> shell(B.kmax + 1, 0.0);
    const int KW = w2_width(B.dim, B.Jmax);
    Tinv.assign(std::max<size_t>((size_t)B.kmax + 1, (size_t)(kW2Off + KW * KW)), 0.0);
    for (auto& o : full) shell[o.q] += std::pow(std::sqrt((double)o.q), expo + 2.0);
    double acc = 0.0;
    for (int64_t k = 0; k <= B.kmax; ++k) {
        acc += shell[k];
        Tinv[k] = acc > 0 ? m2 / acc : 0.0;
    }
    if (B.kmax < KW)
        for (int sh = 1; sh <= B.kmax; ++sh)
            for (int k = sh; k <= B.kmax; ++k)
                Tinv[kW2Off + sh * KW + k] = std::pow(std::sqrt((double)sh), expo) * Tinv[k];
    // after them, the batched kernel's form of the same offsets: the offset
    // of the partner in its staged tile (rows of 64 + 2J, planes of TY + 2J
    // rows; TY = 4 in 3D, 16 in 2D), |z|^2 and the start of the shell's
    // weight row less one (the kernel indexes it by ceil(t) = k_ij + 1), plus
    // a sentinel: no per-offset arithmetic in its pair loop
    const int ngen = (int)fb.size();
    const int J = B.Jmax, pitch = 64 + 2 * J, plane = ((B.dim == 3 ? 4 : 16) + 2 * J) * pitch;
    for (auto& o : full) {
        const int4 bo = box_offset(B.dim, o);
        const int off = (B.dim == 3 ? bo.x * plane : 0) + bo.y * pitch + bo.z;
        fb.push_back(make_int4(off, (int)o.q, (int)o.q * KW - 1, 0));
    }
    fb.push_back(make_int4(0, 1 << 30, 0, 0));
    return ngen;
}

template <typename T>
static int tune_div_batch(Batch& B, const Inst* di, const int2* dit, const T* p, T* q, const int4* full,
                          const double* fw, int nfull, const double* Tinv, hipStream_t s);

template <typename T>
static int cg_solve_t(const ndl_plan* plans, int nprob, const double* const* b, double* const* x,
                      const ndl_cg_opts* opts, ndl_cg_report* reports, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    Batch B;
    std::vector<DevBuf> keep;
    NDL_TRY(build_batch(plans, nprob, B, false, keep));
    const bool mixed = sizeof(T) == 4;
    const int nitems = (int)B.items.size();
    const int64_t tot = B.total;
    // device tables
    DevBuf d_insts, d_items, d_owner, d_full, d_fw, d_Tinv, d_sc;
    NDL_TRY(alloc<Inst>(d_insts, nprob));
    NDL_TRY(alloc<int2>(d_items, nitems));
    NDL_TRY(alloc<int>(d_owner, B.owner.size()));
    NDL_HIP(hipMemcpy(d_insts.p, B.insts.data(), nprob * sizeof(Inst), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_items.p, B.items.data(), nitems * sizeof(int2), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_owner.p, B.owner.data(), B.owner.size() * sizeof(int), hipMemcpyHostToDevice));
    // full ball table sorted by |z|^2, weights |z|^e, and M / T_e[k]
    const Plan& p0 = *reinterpret_cast<const Plan*>(plans[0]);
    std::vector<int4> fb;
    std::vector<double> fwv, Tinv;
    const int nfull = ball_tables(B, p0.expo, p0.m2, fb, fwv, Tinv);
    NDL_TRY(alloc<int4>(d_full, fb.size()));
    NDL_TRY(alloc<double>(d_fw, fwv.size()));
    NDL_TRY(alloc<double>(d_Tinv, Tinv.size()));
    NDL_HIP(hipMemcpy(d_full.p, fb.data(), fb.size() * sizeof(int4), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_fw.p, fwv.data(), fwv.size() * sizeof(double), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_Tinv.p, Tinv.data(), Tinv.size() * sizeof(double), hipMemcpyHostToDevice));
    NDL_TRY(alloc<Scal>(d_sc, nprob));
    NDL_HIP(hipMemset(d_sc.p, 0, nprob * sizeof(Scal)));

    // FP64 fields for the outer residual of FP32 plans
    std::vector<DevBuf> f64f(2 * nprob);
    std::vector<Inst> insts64 = B.insts;
    if (mixed) {
        for (int i = 0; i < nprob; ++i) {
            const Plan& p = *reinterpret_cast<const Plan*>(plans[i]);
            NDL_TRY(alloc<double>(f64f[2 * i], p.N));
            NDL_TRY(alloc<double>(f64f[2 * i + 1], p.N));
            k_widen<float><<<grid_for(p.N), 256, 0, s>>>((const float*)p.prob.delta, (double*)f64f[2 * i].p, p.N);
            k_widen<float><<<grid_for(p.N), 256, 0, s>>>((const float*)p.prob.coef, (double*)f64f[2 * i + 1].p, p.N);
            insts64[i].delta = f64f[2 * i].p;
            insts64[i].coef = f64f[2 * i + 1].p;
        }
    }
    DevBuf d_insts64;
    NDL_TRY(alloc<Inst>(d_insts64, nprob));
    NDL_HIP(hipMemcpy(d_insts64.p, insts64.data(), nprob * sizeof(Inst), hipMemcpyHostToDevice));

    // vectors (concatenated): FP64 b, x, r, ax ; inner T: x_in(d), r, z, p, q, dinv
    DevBuf vb, vx, vr64, vax, vd, vr, vz, vp, vq, vdinv, vdiag64, prz, prr, ppq, pn2, sbn, sres, sscale, sact, stol2;
    NDL_TRY(alloc<double>(vb, tot));
    NDL_TRY(alloc<double>(vx, tot));
    NDL_TRY(alloc<double>(vr64, tot));
    NDL_TRY(alloc<double>(vax, tot));
    NDL_TRY(alloc<T>(vd, tot));
    NDL_TRY(alloc<T>(vr, tot));
    NDL_TRY(alloc<T>(vz, tot));
    NDL_TRY(alloc<T>(vp, tot));
    NDL_TRY(alloc<T>(vq, tot));
    NDL_TRY(alloc<T>(vdinv, tot));
    NDL_TRY(alloc<double>(prz, nitems));
    NDL_TRY(alloc<double>(prr, nitems));
    NDL_TRY(alloc<double>(ppq, nitems));
    NDL_TRY(alloc<double>(pn2, nitems));
    NDL_TRY(alloc<double>(sbn, nprob));
    NDL_TRY(alloc<double>(sres, nprob));
    NDL_TRY(alloc<double>(sscale, nprob));
    NDL_TRY(alloc<int>(sact, nprob));
    NDL_TRY(alloc<double>(stol2, nprob));
    NDL_HIP(hipMemsetAsync(vb.p, 0, tot * sizeof(double), s));
    NDL_HIP(hipMemsetAsync(vx.p, 0, tot * sizeof(double), s));
    for (int i = 0; i < nprob; ++i) {
        NDL_HIP(hipMemcpyAsync((double*)vb.p + B.insts[i].off, b[i], B.insts[i].N * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        NDL_HIP(hipMemcpyAsync((double*)vx.p + B.insts[i].off, x[i], B.insts[i].N * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    }
    const Inst* di = (const Inst*)d_insts.p;
    const Inst* di64 = (const Inst*)d_insts64.p;
    const int2* dit = (const int2*)d_items.p;
    const int* down = (const int*)d_owner.p;
    unsigned gi = (unsigned)std::min(nitems, 256 * 8);
    unsigned gp = (unsigned)((nprob + 63) / 64);
    // the outer FP64 residual of a 3D mixed solve reads the FP32 fields directly
    const bool res32 = mixed && B.dim == 3 && use_div_spec<double>(B, true);
    const Inst* dres = res32 ? di : di64;
    NDL_TRY(prepare_lds<T>(B));
    NDL_TRY(prepare_lds<double>(B, res32));
    // Jacobi: dinv = 1 / diag(-L) (in the inner type)
    NDL_TRY(launch_div_items<T>(B, di, dit, (const T*)nullptr, (T*)vq.p, (const int4*)d_full.p,
                                (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, nullptr, nullptr, true, s));
    k_recip<T><<<grid_for(tot), 256, 0, s>>>((const T*)vq.p, (T*)vdinv.p, tot);
    NDL_HIP(hipGetLastError());
    // launch variant of the apply, timed on this batch (before the graph is captured)
    NDL_TRY(tune_div_batch<T>(B, di, dit, (const T*)vdinv.p, (T*)vq.p, (const int4*)d_full.p,
                              (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, s));

    // ||b||^2 per problem
    NDL_HIP(hipMemsetAsync(vax.p, 0, tot * sizeof(double), s));
    k_residual<T><<<gi, 256, 0, s>>>(di, dit, nitems, (const double*)vb.p, (const double*)vax.p, (double*)vr64.p,
                                      (double*)pn2.p);
    k_item_sums<<<nprob, 256, 0, s>>>(nprob, di, (const double*)pn2.p, (double*)sbn.p);
    std::vector<double> bn2(nprob), res2(nprob);
    NDL_HIP(hipMemcpyAsync(bn2.data(), sbn.p, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
    NDL_HIP(hipStreamSynchronize(s));

    const double rtol = opts && opts->rtol > 0 ? opts->rtol : 1e-8;
    const int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 100000;
    const int G = opts && opts->graph_iters > 0 ? opts->graph_iters : 25;
    const double inner_rtol = opts && opts->inner_rtol > 0 ? opts->inner_rtol : (mixed ? 1e-5 : rtol);
    std::vector<int> iters(nprob, 0), outer(nprob, 0), conv(nprob, 0), active(nprob, 1), broke(nprob, 0);
    std::vector<double> rel(nprob, 1.0);

    // graph of G inner iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    auto one_iter = [&](hipStream_t st) -> int {
        NDL_TRY(launch_div_items<T>(B, di, dit, (const T*)vp.p, (T*)vq.p, (const int4*)d_full.p,
                                    (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, (const Scal*)d_sc.p,
                                    (double*)ppq.p, false, st));
        k_cg_scalars<<<nprob, 256, 0, st>>>(nprob, di, (Scal*)d_sc.p, (const double*)ppq.p, nullptr, 0, max_iter);
        k_cg_update<T><<<gi, 256, 0, st>>>(di, dit, nitems, (const Scal*)d_sc.p, (T*)vd.p, (T*)vr.p, (T*)vz.p,
                                           (const T*)vp.p, (const T*)vq.p, (const T*)vdinv.p, (double*)prz.p,
                                           (double*)prr.p);
        k_cg_scalars<<<nprob, 256, 0, st>>>(nprob, di, (Scal*)d_sc.p, (const double*)prz.p, (const double*)prr.p, 1,
                                         max_iter);
        k_cg_dir<T><<<gi, 256, 0, st>>>(di, dit, nitems, (const Scal*)d_sc.p, (const T*)vz.p, (T*)vp.p);
        NDL_HIP(hipGetLastError());
        return NDL_OK;
    };
    {
        hipStream_t cs;
        NDL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        NDL_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int rc = NDL_OK;
        for (int g = 0; g < G && rc == NDL_OK; ++g) rc = one_iter(cs);
        hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (rc != NDL_OK) { (void)hipStreamDestroy(cs); return rc; }
        NDL_HIP(ce);
        NDL_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        NDL_HIP(hipStreamDestroy(cs));
    }
    std::unique_ptr<std::remove_pointer<hipGraphExec_t>::type, hipError_t (*)(hipGraphExec_t)> gx(gexec,
                                                                                                     hipGraphExecDestroy);
    std::unique_ptr<std::remove_pointer<hipGraph_t>::type, hipError_t (*)(hipGraph_t)> gg(graph, hipGraphDestroy);

    std::vector<Scal> hsc(nprob);
    std::vector<double> scale(nprob), tol2(nprob);
    const int max_outer = mixed ? 20 : 3;
    for (int out_it = 0; out_it < max_outer; ++out_it) {
        // true FP64 residual r = b - A x
        NDL_TRY(launch_div_items<double>(B, dres, dit, (const double*)vx.p, (double*)vax.p, (const int4*)d_full.p,
                                         (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, nullptr, nullptr,
                                         false, s, res32));
        k_residual<double><<<gi, 256, 0, s>>>(di, dit, nitems, (const double*)vb.p, (const double*)vax.p,
                                               (double*)vr64.p, (double*)pn2.p);
        k_item_sums<<<nprob, 256, 0, s>>>(nprob, di, (const double*)pn2.p, (double*)sres.p);
        NDL_HIP(hipMemcpyAsync(res2.data(), sres.p, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
        NDL_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int i = 0; i < nprob; ++i) {
            double bn = std::sqrt(bn2[i]);
            rel[i] = bn > 0 ? std::sqrt(res2[i]) / bn : std::sqrt(res2[i]);
            if (rel[i] <= rtol) { conv[i] = 1; active[i] = 0; }
            else if (iters[i] >= max_iter || broke[i]) active[i] = 0;
            if (active[i]) any = true;
            double rn = std::sqrt(res2[i]);
            scale[i] = rn > 0 ? 1.0 / rn : 1.0;
            // inner target: relative reduction inner_rtol, never below what the outer needs
            double want = mixed ? std::max(inner_rtol, 0.5 * rtol * (bn > 0 ? bn : 1.0) / (rn > 0 ? rn : 1.0))
                                : rtol * (bn > 0 ? bn : 1.0) / (rn > 0 ? rn : 1.0);
            tol2[i] = active[i] ? want * want : 1e300;
        }
        if (!any) break;
        for (int i = 0; i < nprob; ++i) outer[i] += active[i];
        NDL_HIP(hipMemcpyAsync(sscale.p, scale.data(), nprob * sizeof(double), hipMemcpyHostToDevice, s));
        NDL_HIP(hipMemcpyAsync(stol2.p, tol2.data(), nprob * sizeof(double), hipMemcpyHostToDevice, s));
        NDL_HIP(hipMemcpyAsync(sact.p, active.data(), nprob * sizeof(int), hipMemcpyHostToDevice, s));
        // inner right-hand side r / ||r|| in the inner type; d = 0
        k_scale_copy<T, double><<<grid_for(tot), 256, 0, s>>>(di, down, tot, (const double*)vr64.p, (T*)vr.p,
                                                               (const double*)sscale.p);
        k_cg_init<T><<<gi, 256, 0, s>>>(di, dit, nitems, (T*)vd.p, (const T*)vr.p, (T*)vz.p, (T*)vp.p,
                                         (const T*)vdinv.p, (double*)prz.p, (double*)prr.p);
        // reset per-problem scalars; inactive problems start as done
        for (int i = 0; i < nprob; ++i) { hsc[i] = Scal{}; hsc[i].iters = iters[i]; }
        NDL_HIP(hipMemcpyAsync(d_sc.p, hsc.data(), nprob * sizeof(Scal), hipMemcpyHostToDevice, s));
        k_cg_start<<<nprob, 256, 0, s>>>(nprob, di, (Scal*)d_sc.p, (const double*)prz.p, (const double*)prr.p,
                                      (const double*)stol2.p);
        // replay the graph until every active problem has finished its inner solve
        for (;;) {
            NDL_HIP(hipGraphLaunch(gexec, s));
            NDL_HIP(hipMemcpyAsync(hsc.data(), d_sc.p, nprob * sizeof(Scal), hipMemcpyDeviceToHost, s));
            NDL_HIP(hipStreamSynchronize(s));
            bool busy = false;
            for (int i = 0; i < nprob; ++i)
                if (!hsc[i].done) busy = true;
            if (!busy) break;
        }
        for (int i = 0; i < nprob; ++i) {
            if (!active[i]) continue;
            iters[i] = hsc[i].iters;
            if (hsc[i].done == 3) broke[i] = 1;
        }
        // x += ||r|| d (FP64)
        k_axpy_outer<T><<<grid_for(tot), 256, 0, s>>>(down, tot, (double*)vx.p, (const T*)vd.p,
                                                       (const double*)sscale.p, (const int*)sact.p);
        NDL_HIP(hipGetLastError());
    }
    // final residual (FP64) and copy-out
    NDL_TRY(launch_div_items<double>(B, dres, dit, (const double*)vx.p, (double*)vax.p, (const int4*)d_full.p,
                                     (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, nullptr, nullptr, false,
                                     s, res32));
    k_residual<double><<<gi, 256, 0, s>>>(di, dit, nitems, (const double*)vb.p, (const double*)vax.p,
                                           (double*)vr64.p, (double*)pn2.p);
    k_item_sums<<<nprob, 256, 0, s>>>(nprob, di, (const double*)pn2.p, (double*)sres.p);
    NDL_HIP(hipMemcpyAsync(res2.data(), sres.p, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
    for (int i = 0; i < nprob; ++i)
        NDL_HIP(hipMemcpyAsync(x[i], (double*)vx.p + B.insts[i].off, B.insts[i].N * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    NDL_HIP(hipStreamSynchronize(s));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool allc = true;
    for (int i = 0; i < nprob; ++i) {
        double bn = std::sqrt(bn2[i]);
        rel[i] = bn > 0 ? std::sqrt(res2[i]) / bn : std::sqrt(res2[i]);
        conv[i] = rel[i] <= rtol;
        allc = allc && conv[i];
        if (reports) {
            reports[i].iters = iters[i];
            reports[i].outer = outer[i];
            reports[i].converged = conv[i];
            reports[i].fell_back = 0;
            reports[i].rel_res_fp64 = rel[i];
            reports[i].seconds = secs;
        }
    }
    for (int i = 0; i < nprob; ++i)
        if (broke[i] && !conv[i]) {
            set_error("CG broke down on problem %d (non-positive curvature or NaN)", i);
            return NDL_EBREAKDOWN;
        }
    if (!allc) {
        set_error("CG did not reach rtol=%g within the iteration limit on every problem", rtol);
        return NDL_ENOCONV;
    }
    return NDL_OK;
}

// ------------------------------------------------------------------ single-plan operator
// -L on an unpadded vector of one case (b) plan (zero volume constraint),
// with device tables built once and kept by the caller.
struct OpCache {
    const Plan* plan = nullptr;
    uint64_t plan_uid = 0;
    Batch B;
    DevBuf insts, items, full, fw, Tinv, part, sres, dinv;
    int nfull = 0, nitems = 0;
};

// The batch tables of the item kernels for `nprob` plans (one dimension and
// profile): instances, items, the full-ball table and M / T_e[k].
static int op_tables(const ndl_plan* plans, int nprob, OpCache& oc)
{
    std::vector<DevBuf> keep;
    NDL_TRY(build_batch(plans, nprob, oc.B, false, keep));
    const Plan& P = *reinterpret_cast<const Plan*>(plans[0]);
    oc.nitems = (int)oc.B.items.size();
    NDL_TRY(alloc<Inst>(oc.insts, nprob));
    NDL_TRY(alloc<int2>(oc.items, oc.nitems));
    NDL_HIP(hipMemcpy(oc.insts.p, oc.B.insts.data(), nprob * sizeof(Inst), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(oc.items.p, oc.B.items.data(), oc.nitems * sizeof(int2), hipMemcpyHostToDevice));
    std::vector<int4> fb;
    std::vector<double> fwv, Tinv;
    oc.nfull = ball_tables(oc.B, P.expo, P.m2, fb, fwv, Tinv);
    NDL_TRY(alloc<int4>(oc.full, fb.size()));
    NDL_TRY(alloc<double>(oc.fw, fwv.size()));
    NDL_TRY(alloc<double>(oc.Tinv, Tinv.size()));
    NDL_HIP(hipMemcpy(oc.full.p, fb.data(), fb.size() * sizeof(int4), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(oc.fw.p, fwv.data(), fwv.size() * sizeof(double), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(oc.Tinv.p, Tinv.data(), Tinv.size() * sizeof(double), hipMemcpyHostToDevice));
    return NDL_OK;
}

// Autotuner of the batched item kernel: times every launch variant on the
// batch itself (input p, non-zero, output q as scratch) and keeps the fastest
// in B.variant; cached per (dim, reach, element type, batch size class).
template <typename T>
static int tune_div_batch(Batch& B, const Inst* di, const int2* dit, const T* p, T* q, const int4* full,
                          const double* fw, int nfull, const double* Tinv, hipStream_t s)
{
    if (!use_div_spec<T>(B)) return NDL_OK;
    const int nitems = (int)B.items.size();
    int lg = 0;
    while ((1 << (lg + 1)) <= nitems) ++lg;
    const std::string key = "div.d" + std::to_string(B.dim) + ".J" + std::to_string(B.Jmax) + ".t" +
                            std::to_string(sizeof(T)) + ".i" + std::to_string(lg);
    int cached = 0;
    if (tune_cache_lookup(key, &cached) && cached >= 0 && cached < div_num_variants(B.dim)) {
        B.variant = cached;
        return NDL_OK;
    }
    hipEvent_t e0, e1;
    NDL_HIP(hipEventCreate(&e0));
    NDL_HIP(hipEventCreate(&e1));
    const int nv = div_num_variants(B.dim);
    std::vector<float> t(nv, 1e30f);
    int rc = NDL_OK;
    for (int round = 0; round < 2 && rc == NDL_OK; ++round)
        for (int v = 0; v < nv && rc == NDL_OK; ++v) {
            rc = launch_div_items<T>(B, di, dit, p, q, full, fw, nfull, Tinv, nullptr, nullptr, false, s, false, v);
            if (rc != NDL_OK) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 4 && rc == NDL_OK; ++r)
                rc = launch_div_items<T>(B, di, dit, p, q, full, fw, nfull, Tinv, nullptr, nullptr, false, s, false,
                                         v);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t[v] = std::min(t[v], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NDL_OK) return rc;
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (t[v] < t[best]) best = v;
    B.variant = best;
    tune_cache_store(key, best);
    return NDL_OK;
}

template <typename T>
static int op_build(const Plan& P, OpCache& oc, hipStream_t s)
{
    if (oc.plan == &P && oc.plan_uid == P.uid) return NDL_OK;
    oc = OpCache();
    ndl_plan h = reinterpret_cast<ndl_plan>(const_cast<Plan*>(&P));
    NDL_TRY(op_tables(&h, 1, oc));
    NDL_TRY(alloc<double>(oc.part, oc.nitems));
    NDL_TRY(alloc<double>(oc.sres, 2));
    NDL_TRY(alloc<T>(oc.dinv, P.N));
    NDL_TRY(prepare_lds<T>(oc.B));
    NDL_TRY(launch_div_items<T>(oc.B, (const Inst*)oc.insts.p, (const int2*)oc.items.p, (const T*)nullptr,
                                (T*)oc.dinv.p, (const int4*)oc.full.p, (const double*)oc.fw.p, oc.nfull,
                                (const double*)oc.Tinv.p, nullptr, nullptr, true, s));
    k_recip<T><<<grid_for(P.N), 256, 0, s>>>((const T*)oc.dinv.p, (T*)oc.dinv.p, P.N);
    NDL_HIP(hipGetLastError());
    {
        // tune the apply on the diagonal's inverse (a non-zero field) into a scratch output
        DevBuf scr;
        NDL_TRY(alloc<T>(scr, P.N));
        NDL_TRY(tune_div_batch<T>(oc.B, (const Inst*)oc.insts.p, (const int2*)oc.items.p, (const T*)oc.dinv.p,
                                  (T*)scr.p, (const int4*)oc.full.p, (const double*)oc.fw.p, oc.nfull,
                                  (const double*)oc.Tinv.p, s));
        NDL_HIP(hipStreamSynchronize(s));
    }
    oc.plan = &P;
    oc.plan_uid = P.uid;
    return NDL_OK;
}

static OpCache g_op_cache;  // one cached operator (the training loop uses one plan at a time)

// y = -L x (unpadded, FP32) for one plan; dinv = 1 / diag(-L) available after the call
int plan_neg_L_f32(const Plan& P, const float* x, float* y, const float** dinv, hipStream_t s)
{
    if (P.form != NDL_DIV || P.prec == NDL_F64) {
        set_error("internal: FP32 case (b) plan expected");
        return NDL_EINVAL;
    }
    NDL_TRY(op_build<float>(P, g_op_cache, s));
    OpCache& oc = g_op_cache;
    NDL_TRY(launch_div_items<float>(oc.B, (const Inst*)oc.insts.p, (const int2*)oc.items.p, x, y,
                                    (const int4*)oc.full.p, (const double*)oc.fw.p, oc.nfull,
                                    (const double*)oc.Tinv.p, nullptr, nullptr, false, s));
    if (dinv) *dinv = (const float*)oc.dinv.p;
    return NDL_OK;
}

int plan_dinv_f32(const Plan& P, const float** dinv, hipStream_t s)
{
    if (P.form != NDL_DIV || P.prec == NDL_F64) {
        set_error("internal: FP32 case (b) plan expected");
        return NDL_EINVAL;
    }
    NDL_TRY(op_build<float>(P, g_op_cache, s));
    *dinv = (const float*)g_op_cache.dinv.p;
    return NDL_OK;
}

// ------------------------------------------------------------------ flexible PCG with M(r)
template <typename T>
__global__ void k_dot2(const Inst* __restrict__ insts, const int2* __restrict__ items, int nitems,
                       const T* __restrict__ r, const T* __restrict__ a, const T* __restrict__ b,
                       double* __restrict__ pa, double* __restrict__ pb)
{
    __shared__ double red[4];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        double s1 = 0.0, s2 = 0.0;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            double rv = (double)r[gi];
            s1 += rv * (double)a[gi];
            if (b) s2 += rv * (double)b[gi];
        }
        double t1 = block_sum(s1, red);
        double t2 = block_sum(s2, red);
        if (threadIdx.x == 0) { pa[it] = t1; if (pb) pb[it] = t2; }
    }
}

// Device scalars of the flexible PCG inner solve (one problem):
//   [0] alpha  [1] p.q  [2] breakdown flag (p.q <= 0 or not finite)
//   [3] r.r    [4] (written with r.r, unused)
//   [5] r.z of the current direction  [6] beta
//   [7] flag: the last r.z was not positive or not finite
constexpr int kLpcgScalars = 8;

// p = z + beta p ; z_old = z (skipped while the r.z flag is set: the host
// recomputes z by Jacobi first)
template <typename T>
__global__ void k_dir2(int64_t n, const double* __restrict__ sc, const T* __restrict__ z, T* __restrict__ p,
                       T* __restrict__ zold)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || sc[7] != 0.0) return;
    const T beta = (T)sc[6];
    T zv = z[i];
    p[i] = zv + beta * p[i];
    zold[i] = zv;
}

// alpha = r.z / p.q (items summed in the fixed order).  A breakdown, or a
// pending r.z flag, gives alpha = 0 (d and r stay as they are); only the
// former raises the breakdown flag.
__global__ void k_pq_alpha(const Inst* __restrict__ insts, const double* __restrict__ part, double* __restrict__ sc)
{
    __shared__ double sh[256];
    const Inst I = insts[0];
    const double pq = problem_sum(I, part, sh);
    if (threadIdx.x != 0) return;
    const bool pending = sc[7] != 0.0;
    const bool ok = pq > 0.0 && isfinite(pq);
    sc[0] = (ok && !pending) ? sc[5] / pq : 0.0;
    sc[1] = pq;
    sc[2] = (ok || pending) ? 0.0 : 1.0;
}

// r.z_new and r.z_old from the item partials -> the Polak-Ribiere beta
// (clipped at 0) and the new r.z; restart = 1 only sets r.z (a new first
// direction p = z).  A non-positive or non-finite r.z raises flag [7] and
// leaves r.z and beta unchanged.
__global__ void k_lpcg_beta(const Inst* __restrict__ insts, const double* __restrict__ pa,
                            const double* __restrict__ pb, double* __restrict__ sc, int restart)
{
    __shared__ double sh[256];
    const Inst I = insts[0];
    const double rzn = problem_sum(I, pa, sh);
    const double rzo = restart ? 0.0 : problem_sum(I, pb, sh);
    if (threadIdx.x != 0) return;
    if (!(rzn > 0.0) || !isfinite(rzn)) {
        sc[7] = 1.0;
        return;
    }
    if (!restart) {
        double beta = (rzn - rzo) / sc[5];
        sc[6] = beta >= 0.0 ? beta : 0.0;
    }
    sc[5] = rzn;
    sc[7] = 0.0;
}

// d += alpha p, r -= alpha q over one problem's items, with the per-item
// partials of r.r (alpha read from the device)
template <typename T>
__global__ __launch_bounds__(256) void k_axpy2_rr(const Inst* __restrict__ insts, const int2* __restrict__ items,
                                                  int nitems, const double* __restrict__ alpha, T* __restrict__ d,
                                                  T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                                                  double* __restrict__ prr)
{
    __shared__ double red[4];
    const T a = (T)alpha[0];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int2 item = items[it];
        const Inst I = insts[item.x];
        int org[3];
        item_geom<T>(I, item.y, org);
        int ext[3] = {I.dim >= 3 ? I.n : 1, I.dim >= 2 ? I.n : 1, I.n};
        double s1 = 0.0;
        int npts = I.E[0] * I.E[1] * I.E[2];
        for (int pi = threadIdx.x; pi < npts; pi += blockDim.x) {
            int e2 = pi % I.E[2];
            int rr_ = pi / I.E[2];
            int e1 = rr_ % I.E[1];
            int e0 = rr_ / I.E[1];
            int x0 = org[0] + e0, x1 = org[1] + e1, x2 = org[2] + e2;
            if (!(x0 < ext[0] && x1 < ext[1] && x2 < ext[2])) continue;
            int64_t gi = I.off + ((int64_t)x0 * ext[1] + x1) * ext[2] + x2;
            d[gi] += a * p[gi];
            const T rv = r[gi] - a * q[gi];
            r[gi] = rv;
            s1 += (double)rv * (double)rv;
        }
        double t1 = block_sum(s1, red);
        if (threadIdx.x == 0) prr[it] = t1;
    }
}

// the sums of two item-partial arrays of one problem: out[0], out[1]
__global__ void k_item_sums2(const Inst* __restrict__ insts, const double* __restrict__ pa,
                             const double* __restrict__ pb, double* __restrict__ out)
{
    __shared__ double sh[256];
    const Inst I = insts[0];
    const double a = problem_sum(I, pa, sh);
    const double b = pb ? problem_sum(I, pb, sh) : 0.0;
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// z = r / diag (+ z when add)
template <typename T>
__global__ void k_jacobi_add(int64_t n, const T* __restrict__ r, const T* __restrict__ dinv, T* __restrict__ z, int add)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = r[i] * dinv[i] + (add ? z[i] : T(0));
}

// One problem; the inner solve uses z = M(r) from the network (flexible CG,
// Polak-Ribiere beta).  A breakdown (p.q <= 0, r.z <= 0, non-finite values)
// switches the rest of the solve to Jacobi (reported as fell_back).
template <typename T>
static int pcg_learned_t(const ndl_plan plan, const double* b, double* x, const ndl_cg_opts* opts,
                         ndl_cg_report* rep, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const Plan& P = *reinterpret_cast<const Plan*>(plan);
    Batch B;
    std::vector<DevBuf> keep;
    NDL_TRY(build_batch(&plan, 1, B, false, keep));
    const int nitems = (int)B.items.size();
    const int64_t N = P.N;
    DevBuf d_insts, d_insts64, d_items, d_full, d_fw, d_Tinv;
    NDL_TRY(alloc<Inst>(d_insts, 1));
    NDL_TRY(alloc<Inst>(d_insts64, 1));
    NDL_TRY(alloc<int2>(d_items, nitems));
    NDL_HIP(hipMemcpy(d_insts.p, B.insts.data(), sizeof(Inst), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_items.p, B.items.data(), nitems * sizeof(int2), hipMemcpyHostToDevice));
    std::vector<int4> fb;
    std::vector<double> fwv, Tinv;
    const int nfull = ball_tables(B, P.expo, P.m2, fb, fwv, Tinv);
    NDL_TRY(alloc<int4>(d_full, fb.size()));
    NDL_TRY(alloc<double>(d_fw, fwv.size()));
    NDL_TRY(alloc<double>(d_Tinv, Tinv.size()));
    NDL_HIP(hipMemcpy(d_full.p, fb.data(), fb.size() * sizeof(int4), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_fw.p, fwv.data(), fwv.size() * sizeof(double), hipMemcpyHostToDevice));
    NDL_HIP(hipMemcpy(d_Tinv.p, Tinv.data(), Tinv.size() * sizeof(double), hipMemcpyHostToDevice));
    // FP64 fields for the outer residual
    DevBuf dd64, dc64;
    Inst i64 = B.insts[0];
    if (sizeof(T) == 4) {
        NDL_TRY(alloc<double>(dd64, N));
        NDL_TRY(alloc<double>(dc64, N));
        k_widen<float><<<grid_for(N), 256, 0, s>>>((const float*)P.prob.delta, (double*)dd64.p, N);
        k_widen<float><<<grid_for(N), 256, 0, s>>>((const float*)P.prob.coef, (double*)dc64.p, N);
        i64.delta = dd64.p;
        i64.coef = dc64.p;
    }
    NDL_HIP(hipMemcpy(d_insts64.p, &i64, sizeof(Inst), hipMemcpyHostToDevice));
    const Inst* di = (const Inst*)d_insts.p;
    const Inst* di64 = (const Inst*)d_insts64.p;
    const int2* dit = (const int2*)d_items.p;
    // the outer FP64 residual of a 3D mixed solve reads the FP32 fields directly
    const bool res32 = sizeof(T) == 4 && B.dim == 3 && use_div_spec<double>(B, true);
    const Inst* dres = res32 ? di : di64;
    NDL_TRY(prepare_lds<T>(B));
    NDL_TRY(prepare_lds<double>(B, res32));
    DevBuf vx, vax, vr64, vd, vr, vz, vzo, vp, vq, vdinv, pa, pb, sres;
    NDL_TRY(alloc<double>(vx, N));
    NDL_TRY(alloc<double>(vax, N));
    NDL_TRY(alloc<double>(vr64, N));
    NDL_TRY(alloc<T>(vd, N));
    NDL_TRY(alloc<T>(vr, N));
    NDL_TRY(alloc<T>(vz, N));
    NDL_TRY(alloc<T>(vzo, N));
    NDL_TRY(alloc<T>(vp, N));
    NDL_TRY(alloc<T>(vq, N));
    NDL_TRY(alloc<T>(vdinv, N));
    NDL_TRY(alloc<double>(pa, nitems));
    NDL_TRY(alloc<double>(pb, nitems));
    NDL_TRY(alloc<double>(sres, 2));
    DevBuf scal;  // the inner solve's device scalars (k_pq_alpha, k_lpcg_beta)
    NDL_TRY(alloc<double>(scal, kLpcgScalars));
    NDL_HIP(hipMemcpyAsync(vx.p, x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    NDL_TRY(launch_div_items<T>(B, di, dit, (const T*)nullptr, (T*)vq.p, (const int4*)d_full.p, (const double*)d_fw.p,
                                nfull, (const double*)d_Tinv.p, nullptr, nullptr, true, s));
    k_recip<T><<<grid_for(N), 256, 0, s>>>((const T*)vq.p, (T*)vdinv.p, N);
    NDL_TRY(tune_div_batch<T>(B, di, dit, (const T*)vdinv.p, (T*)vq.p, (const int4*)d_full.p,
                              (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, s));
    unsigned gi = (unsigned)std::min(nitems, 256 * 8);
    auto sum_items = [&](const double* part, double* out) -> int {
        k_item_sums<<<1, 256, 0, s>>>(1, di, part, (double*)sres.p);
        NDL_HIP(hipMemcpyAsync(out, sres.p, sizeof(double), hipMemcpyDeviceToHost, s));
        NDL_HIP(hipStreamSynchronize(s));
        return NDL_OK;
    };
    // r.z (and r.z_old) into the device scalars: restart = 1 starts a new
    // first direction (r.z only), else beta as well
    auto dots = [&](const T* r, const T* z, const T* zo, int restart) -> int {
        k_dot2<T><<<gi, 256, 0, s>>>(di, dit, nitems, r, z, zo, (double*)pa.p, (double*)pb.p);
        k_lpcg_beta<<<1, 256, 0, s>>>(di, (const double*)pa.p, (const double*)pb.p, (double*)scal.p, restart);
        NDL_HIP(hipGetLastError());
        return NDL_OK;
    };
    auto read_scalars = [&](double* h) -> int {
        NDL_HIP(hipMemcpyAsync(h, scal.p, kLpcgScalars * sizeof(double), hipMemcpyDeviceToHost, s));
        NDL_HIP(hipStreamSynchronize(s));
        return NDL_OK;
    };
    // two-level preconditioner: z = D^-1 r + M(r); the network supplies the
    // smooth part of the correction that the Jacobi term misses
    // (a linear network adds the Jacobi term while unscaling its output)
    const bool fused_jacobi = net_is_linear(opts->net);
    auto precond = [&](const T* r, T* z, bool jac) -> int {
        if (!jac && fused_jacobi) return net_precond(opts->net, P, r, z, s, vdinv.p, true);
        if (!jac) NDL_TRY(net_precond(opts->net, P, r, z, s, vdinv.p));
        k_jacobi_add<T><<<grid_for(N), 256, 0, s>>>(N, r, (const T*)vdinv.p, z, jac ? 0 : 1);
        NDL_HIP(hipGetLastError());
        return NDL_OK;
    };
    // ||b||
    NDL_HIP(hipMemsetAsync(vax.p, 0, N * sizeof(double), s));
    k_residual<double><<<gi, 256, 0, s>>>(di, dit, nitems, b, (const double*)vax.p, (double*)vr64.p, (double*)pa.p);
    double bn2 = 0.0;
    NDL_TRY(sum_items((const double*)pa.p, &bn2));
    const double bn = std::sqrt(bn2);
    const double rtol = opts->rtol > 0 ? opts->rtol : 1e-8;
    const int max_iter = opts->max_iter > 0 ? opts->max_iter : 100000;
    const double inner_rtol = opts->inner_rtol > 0 ? opts->inner_rtol : (sizeof(T) == 4 ? 1e-5 : rtol);
    int iters = 0, outer = 0;
    bool jac = false, conv = false;
    double rel = 1.0;
    // one problem: every node belongs to problem 0; its outer scale 1/||r||
    // and active flag live on the device for the whole solve
    DevBuf down, dsc, dact;
    {
        std::vector<int> own((N + 1023) / 1024, 0);
        const int one = 1;
        NDL_TRY(alloc<int>(down, own.size()));
        NDL_TRY(alloc<double>(dsc, 1));
        NDL_TRY(alloc<int>(dact, 1));
        NDL_HIP(hipMemcpy(down.p, own.data(), own.size() * sizeof(int), hipMemcpyHostToDevice));
        NDL_HIP(hipMemcpy(dact.p, &one, sizeof(int), hipMemcpyHostToDevice));
    }
    double sc = 1.0;  // host copy of the scale sent for the current outer step
    for (int o = 0; o < 20; ++o) {
        NDL_TRY(launch_div_items<double>(B, dres, dit, (const double*)vx.p, (double*)vax.p, (const int4*)d_full.p,
                                         (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, nullptr, nullptr,
                                         false, s, res32));
        k_residual<double><<<gi, 256, 0, s>>>(di, dit, nitems, b, (const double*)vax.p, (double*)vr64.p,
                                               (double*)pa.p);
        double rn2 = 0.0;
        NDL_TRY(sum_items((const double*)pa.p, &rn2));
        rel = bn > 0 ? std::sqrt(rn2) / bn : std::sqrt(rn2);
        if (rel <= rtol) { conv = true; break; }
        if (iters >= max_iter) break;
        ++outer;
        const double rn = std::sqrt(rn2);
        const double want = std::max(inner_rtol, 0.5 * rtol * bn / rn);
        // inner: -L d = r / ||r||
        sc = 1.0 / rn;
        NDL_HIP(hipMemcpyAsync(dsc.p, &sc, sizeof(double), hipMemcpyHostToDevice, s));
        k_scale_copy<T, double><<<grid_for(N), 256, 0, s>>>(di, (const int*)down.p, N, (const double*)vr64.p,
                                                             (T*)vr.p, (const double*)dsc.p);
        NDL_HIP(hipMemsetAsync(vd.p, 0, N * sizeof(T), s));
        NDL_TRY(precond((const T*)vr.p, (T*)vz.p, jac));
        // first direction p = z; a non-positive r.z from the network falls
        // back to Jacobi for the rest of the solve
        double hs[kLpcgScalars];
        NDL_TRY(dots((const T*)vr.p, (const T*)vz.p, nullptr, 1));
        NDL_TRY(read_scalars(hs));
        if (hs[7] != 0.0 && !jac) {
            jac = true;
            NDL_TRY(precond((const T*)vr.p, (T*)vz.p, true));
            NDL_TRY(dots((const T*)vr.p, (const T*)vz.p, nullptr, 1));
        }
        // restart from the current r with the Jacobi preconditioner
        auto restart_jacobi = [&]() -> int {
            jac = true;
            NDL_TRY(precond((const T*)vr.p, (T*)vz.p, true));
            NDL_TRY(dots((const T*)vr.p, (const T*)vz.p, nullptr, 1));
            NDL_HIP(hipMemcpyAsync(vp.p, vz.p, N * sizeof(T), hipMemcpyDeviceToDevice, s));
            NDL_HIP(hipMemcpyAsync(vzo.p, vz.p, N * sizeof(T), hipMemcpyDeviceToDevice, s));
            return NDL_OK;
        };
        NDL_HIP(hipMemcpyAsync(vp.p, vz.p, N * sizeof(T), hipMemcpyDeviceToDevice, s));
        NDL_HIP(hipMemcpyAsync(vzo.p, vz.p, N * sizeof(T), hipMemcpyDeviceToDevice, s));
        double best = 1.0;
        int since_best = 0;
        while (iters < max_iter) {
            // q = A p with the item partials of p.q; alpha, the update and r.r
            // on the device; one read-back per iteration
            NDL_TRY(launch_div_items<T>(B, di, dit, (const T*)vp.p, (T*)vq.p, (const int4*)d_full.p,
                                        (const double*)d_fw.p, nfull, (const double*)d_Tinv.p, nullptr, (double*)pa.p,
                                        false, s));
            k_pq_alpha<<<1, 256, 0, s>>>(di, (const double*)pa.p, (double*)scal.p);
            k_axpy2_rr<T><<<gi, 256, 0, s>>>(di, dit, nitems, (const double*)scal.p, (T*)vd.p, (T*)vr.p,
                                             (const T*)vp.p, (const T*)vq.p, (double*)pb.p);
            k_item_sums2<<<1, 256, 0, s>>>(di, (const double*)pb.p, nullptr, (double*)scal.p + 3);
            NDL_TRY(read_scalars(hs));
            if (hs[7] != 0.0) {
                // the previous iteration's r.z was not positive: its direction
                // update and this iteration's step were skipped (alpha = 0);
                // recompute z by Jacobi and take the update with it
                if (jac) break;
                jac = true;
                NDL_TRY(precond((const T*)vr.p, (T*)vz.p, true));
                NDL_TRY(dots((const T*)vr.p, (const T*)vz.p, (const T*)vzo.p, 0));
                k_dir2<T><<<grid_for(N), 256, 0, s>>>(N, (const double*)scal.p, (const T*)vz.p, (T*)vp.p,
                                                      (T*)vzo.p);
                NDL_HIP(hipGetLastError());
                continue;
            }
            ++iters;
            if (hs[2] != 0.0) {
                if (jac) break;  // even Jacobi broke down: stop this inner solve
                NDL_TRY(restart_jacobi());  // fall back and restart the inner directions
                continue;
            }
            const double rr = hs[3];
            if (std::sqrt(rr) <= want || !std::isfinite(rr)) break;
            // stagnation of the learned directions (no 0.1% drop of the residual
            // in 200 iterations; CG residuals may plateau for a while): fall
            // back to Jacobi
            if (rr < 0.999 * best) { best = rr; since_best = 0; }
            else if (++since_best > 200 && !jac) {
                NDL_TRY(restart_jacobi());
                continue;
            }
            NDL_TRY(precond((const T*)vr.p, (T*)vz.p, jac));
            NDL_TRY(dots((const T*)vr.p, (const T*)vz.p, (const T*)vzo.p, 0));
            k_dir2<T><<<grid_for(N), 256, 0, s>>>(N, (const double*)scal.p, (const T*)vz.p, (T*)vp.p, (T*)vzo.p);
            NDL_HIP(hipGetLastError());
        }
        // x += ||r|| d
        k_axpy_outer<T><<<grid_for(N), 256, 0, s>>>((const int*)down.p, N, (double*)vx.p, (const T*)vd.p,
                                                     (const double*)dsc.p, (const int*)dact.p);
        NDL_HIP(hipGetLastError());
    }
    NDL_HIP(hipMemcpyAsync(x, vx.p, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    NDL_HIP(hipStreamSynchronize(s));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) {
        rep->iters = iters;
        rep->outer = outer;
        rep->converged = conv;
        rep->fell_back = jac;
        rep->rel_res_fp64 = rel;
        rep->seconds = secs;
    }
    if (!conv) {
        set_error("learned PCG did not reach rtol=%g (rel. residual %g)", rtol, rel);
        return NDL_ENOCONV;
    }
    return NDL_OK;
}

}  // namespace ndl

extern "C" {
int ndl_cg_solve(const ndl_plan* plans, int nprob, const double* const* b, double* const* x, const ndl_cg_opts* opts,
                 ndl_cg_report* reports, void* stream)
{
    using namespace ndl;
    if (!plans || nprob <= 0 || !b || !x) { set_error("ndl_cg_solve: bad arguments"); return NDL_EINVAL; }
    const Plan* p0 = reinterpret_cast<const Plan*>(plans[0]);
    if (p0 && p0->form == NDL_SYM) {
        for (int i = 0; i < nprob; ++i) {
            const Plan* p = reinterpret_cast<const Plan*>(plans[i]);
            if (!p || !b[i] || !x[i] || p->form != NDL_SYM) {
                set_error("ndl_cg_solve: plans of the kernel-averaged form and vectors expected (problem %d)", i);
                return NDL_EINVAL;
            }
        }
        if (opts && opts->precond != 0) { set_error("the kernel-averaged form runs Jacobi-CG"); return NDL_EUNSUPPORTED; }
        return sym_cg_solve(plans, nprob, b, x, opts, reports, (hipStream_t)stream);
    }
    for (int i = 0; i < nprob; ++i) {
        const Plan* p = reinterpret_cast<const Plan*>(plans[i]);
        if (!p || !b[i] || !x[i]) { set_error("ndl_cg_solve: null plan or vector %d", i); return NDL_EINVAL; }
        if (p->form != NDL_DIV || p->model != NDL_DIFFUSION) {
            set_error("ndl_cg_solve needs case (b) diffusion plans (case (a) is not symmetric)");
            return NDL_ENOTSPD;
        }
        if (p->kernel == NDL_G_POLY) { set_error("ndl_cg_solve: power profiles only"); return NDL_EUNSUPPORTED; }
        if (p->dim != p0->dim || (p->prec == NDL_F64) != (p0->prec == NDL_F64) || p->kernel != p0->kernel ||
            p->expo != p0->expo || p->m2 != p0->m2 || p->norm != p0->norm) {
            set_error("ndl_cg_solve: all plans of one call must share dim, precision class and kernel");
            return NDL_EINVAL;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (opts && opts->precond == 1) {
        if (!opts->net) { set_error("precond = 1 needs opts->net"); return NDL_EINVAL; }
        if (nprob != 1 || p0->dim != 3 || p0->n % 8 != 0) {
            set_error("learned PCG runs one 3D problem with n divisible by 8 per call");
            return NDL_EUNSUPPORTED;
        }
        return p0->prec == NDL_F64 ? pcg_learned_t<double>(plans[0], b[0], x[0], opts, reports, s)
                                   : pcg_learned_t<float>(plans[0], b[0], x[0], opts, reports, s);
    }
    return p0->prec == NDL_F64 ? cg_solve_t<double>(plans, nprob, b, x, opts, reports, s)
                               : cg_solve_t<float>(plans, nprob, b, x, opts, reports, s);
}

}  // extern "C"

namespace ndl {
template <typename T>
static int div_batch_apply_t(const ndl_plan* plans, int nprob, const void* const* x, void* const* y, int variant,
                             int* used, int* nv, hipStream_t s)
{
    OpCache oc;
    NDL_TRY(op_tables(plans, nprob, oc));
    Batch& B = oc.B;
    const bool spec = use_div_spec<T>(B);
    const int nvar = spec ? div_num_variants(B.dim) : 1;
    if (nv) *nv = nvar;
    if (variant >= nvar) {
        set_error("ndl_div_batch_apply: variant %d out of range [0, %d)", variant, nvar);
        return NDL_EINVAL;
    }
    DevBuf vin, vout;
    NDL_TRY(alloc<T>(vin, B.total));
    NDL_TRY(alloc<T>(vout, B.total));
    NDL_HIP(hipMemsetAsync(vin.p, 0, B.total * sizeof(T), s));
    for (int i = 0; i < nprob; ++i)
        NDL_HIP(hipMemcpyAsync((T*)vin.p + B.insts[i].off, x[i], B.insts[i].N * sizeof(T), hipMemcpyDeviceToDevice, s));
    NDL_TRY(prepare_lds<T>(B));
    const Inst* di = (const Inst*)oc.insts.p;
    const int2* dit = (const int2*)oc.items.p;
    if (variant < 0)
        NDL_TRY(tune_div_batch<T>(B, di, dit, (const T*)vin.p, (T*)vout.p, (const int4*)oc.full.p,
                                  (const double*)oc.fw.p, oc.nfull, (const double*)oc.Tinv.p, s));
    else
        B.variant = variant;
    NDL_TRY(launch_div_items<T>(B, di, dit, (const T*)vin.p, (T*)vout.p, (const int4*)oc.full.p,
                                (const double*)oc.fw.p, oc.nfull, (const double*)oc.Tinv.p, nullptr, nullptr, false,
                                s));
    for (int i = 0; i < nprob; ++i)
        NDL_HIP(hipMemcpyAsync(y[i], (const T*)vout.p + B.insts[i].off, B.insts[i].N * sizeof(T),
                               hipMemcpyDeviceToDevice, s));
    NDL_HIP(hipStreamSynchronize(s));
    if (used) *used = spec ? B.variant : 0;
    return NDL_OK;
}
}  // namespace ndl

extern "C" {
int ndl_div_batch_apply(const ndl_plan* plans, int nprob, const void* const* x, void* const* y, int variant,
                        int* variant_used, int* nvariants, void* stream)
{
    using namespace ndl;
    if (!plans || nprob <= 0 || !x || !y) { set_error("ndl_div_batch_apply: bad arguments"); return NDL_EINVAL; }
    const Plan* p0 = reinterpret_cast<const Plan*>(plans[0]);
    for (int i = 0; i < nprob; ++i) {
        const Plan* p = reinterpret_cast<const Plan*>(plans[i]);
        if (!p || !x[i] || !y[i]) { set_error("ndl_div_batch_apply: null plan or vector %d", i); return NDL_EINVAL; }
        if (p->form != NDL_DIV || p->model != NDL_DIFFUSION || p->kernel > NDL_G_FRAC) {
            set_error("ndl_div_batch_apply: case (b) diffusion plans with a power profile");
            return NDL_EUNSUPPORTED;
        }
        if (p->dim != p0->dim || (p->prec == NDL_F64) != (p0->prec == NDL_F64) || p->kernel != p0->kernel ||
            p->expo != p0->expo || p->m2 != p0->m2 || p->norm != p0->norm) {
            set_error("ndl_div_batch_apply: all plans must share dim, precision class and kernel");
            return NDL_EINVAL;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    return p0->prec == NDL_F64 ? div_batch_apply_t<double>(plans, nprob, x, y, variant, variant_used, nvariants, s)
                               : div_batch_apply_t<float>(plans, nprob, x, y, variant, variant_used, nvariants, s);
}


}
