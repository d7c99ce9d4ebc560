/*
 * ndl.h -- C ABI of the MI355X (gfx950) library for nonlocal operators with a
 * finite interaction distance (Tian & Engquist, arXiv 1905.08375).
 *
 * The operator, on Omega = [0,1]^dim with n nodes per axis (h = 1/n, node i at
 * (i+1/2)h), is the quadrature of eq. "eq:diffusion" (Section 2):
 *
 *     L u(x_i) = sum_{0 < |z|^2 <= k_i} omega_i(z) (u(x_i + z h) - u(x_i)) h^dim,
 *     omega_i(z) = C * A * g(|z| / m),   m = delta * n,
 *     k = ceil((delta*n)*(delta*n)) - 1  (evaluated in FP64: the strict ball |y-x| < delta),
 *
 * with the profile g and the constant A chosen by the problem descriptor.  The
 * peridynamic model replaces (u(y)-u(x)) by [e.(u(y)-u(x))] e, e = z/|z| (the
 * linear bond force of Section 1).  Form NDL_ND is case (a) of Section 2
 * (C = c(x), delta = delta(x)); NDL_DIV is case (b) with the symmetric
 * C = (c_i+c_j)/2, delta = (delta_i+delta_j)/2, whose negative is SPD and is
 * the operator the CG solver inverts.
 *
 * Conventions shared by every call
 *  - Every function returns NDL_OK (0) or a negative NDL_E* code and never
 *    aborts; ndl_last_error() gives a message for the calling thread.
 *  - Device buffers (u, Lu, delta, coef, b, x, r, z) are allocated and owned
 *    by the caller; the library never frees or keeps them, except that a plan
 *    keeps the delta/coef pointers of its problem, which must outlive it.
 *  - Plans and nets are opaque, library-owned; destroy them explicitly.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Plan
 *    creation synchronises that stream; applies are asynchronous and
 *    stream-ordered; ndl_cg_solve and ndl_net_train_step return after the
 *    stream has drained (they fill host-side reports).
 *  - Layouts are C order with the last axis fastest.  A state u is the padded
 *    box [batch][ncomp][(n+2R)^dim] whose collar of width R = collar holds the
 *    volume-constraint data (zero for the Dirichlet problem of Section 3);
 *    outputs are [batch][ncomp][n^dim].  ncomp = dim for peridynamics
 *    (component a is the displacement along axis a), else 1.
 *  - Element type follows prec: NDL_F64 = double everywhere; NDL_F32C and
 *    NDL_F32K = float storage with compensated accumulation inside the sums.
 */
#ifndef NDL_H
#define NDL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NDL_OK = 0,
    NDL_EINVAL = -1,       /* bad argument, shape, or collar narrower than the horizon */
    NDL_ENOMEM = -2,       /* device or host allocation failed */
    NDL_EUNSUPPORTED = -3, /* valid but not implemented combination */
    NDL_ENOTSPD = -4,      /* CG asked for a non-symmetric (case (a)) operator */
    NDL_ENOCONV = -5,      /* a solve hit its iteration limit */
    NDL_EHIP = -6,         /* a HIP runtime call failed */
    NDL_EBREAKDOWN = -7    /* preconditioned CG broke down (NaN, r.z <= 0) */
};

/* NDL_F32C: FP32 storage; sums compensated by carrying them in FP64 (FP32
 * pairs add exactly in FP64).  NDL_F32K: FP32 storage and FP32 arithmetic
 * with Kahan-compensated accumulation. */
typedef enum { NDL_F64 = 0, NDL_F32C = 1, NDL_F32K = 2 } ndl_prec;
typedef enum { NDL_DIFFUSION = 0, NDL_PERIDYNAMIC = 1 } ndl_model; /* PD: dim 2 or 3 */
/* Section 2 cases (a), (b); NDL_SYM: the kernel-averaged symmetric form
 * omega_s(x,y) = (omega_x(y) + omega_y(x))/2 of the case (a) weights (a
 * collar partner keeps omega_x), whose negative is SPD; power profiles. */
typedef enum { NDL_ND = 0, NDL_DIV = 1, NDL_SYM = 2 } ndl_form;
/* Radial profile g(r), r = |y-x|/delta:  CONST 1 (the p^0 of Section 3);
 * INV_R 1/r and CONE (1 - r)/r (the two micromoduli of eq. "kernelgamma");
 * FRAC r^-(dim+2s) (fractional micromodulus, Section 1); POLY
 * sum_j poly[j] r^(2j) (the even p^{2K} of Section 3).  Case (b) takes the
 * power profiles CONST, INV_R, FRAC; the hierarchical path all but CONE. */
typedef enum { NDL_G_CONST = 0, NDL_G_INV_R = 1, NDL_G_FRAC = 2, NDL_G_POLY = 3, NDL_G_CONE = 4 } ndl_kernel;
/* Constant A: DISCRETE makes the lattice second moment equal m2_target, so
 * L|x|^2 = 2 dim c exactly (the local limit C Delta u of case (a));
 * CONTINUOUS does the same for the integral over the ball; NONE is the bare
 * 1/delta^(dim+2) of eq. "kernel" (the operator of Example 1). */
typedef enum { NDL_NORM_DISCRETE = 0, NDL_NORM_CONTINUOUS = 1, NDL_NORM_NONE = 2 } ndl_norm;

typedef struct {
    int32_t dim;          /* 1, 2 or 3 */
    int64_t n;            /* nodes per axis, >= 1 */
    int32_t collar;       /* R: padding of u; must satisfy k_max <= (R+1)^2 - 1 */
    int32_t model;        /* ndl_model */
    int32_t form;         /* ndl_form */
    int32_t kernel;       /* ndl_kernel */
    double s;             /* FRAC order, 0 <= s < 1 */
    int32_t K;            /* POLY degree 2K, coefficients poly[0..K] (host pointer, copied) */
    const double* poly;
    int32_t norm;         /* ndl_norm */
    double m2_target;     /* 0 => 2 dim (diffusion) or 2 dim (dim+2) (peridynamics) */
    int32_t prec;         /* ndl_prec */
    const void* delta;    /* device, n^dim horizons (element type of prec), > 0 */
    const void* coef;     /* device, n^dim coefficients c(x) (element type of prec) */
} ndl_problem;

typedef struct ndl_plan_s* ndl_plan;

/* Plan: validates the problem, computes per node the integer cutoff k_i and
 * the scale of the operator from (delta, coef) in FP64, checks the collar, and
 * picks the kernel variant (the autotuner's cached tile, see
 * ndl_autotune).  With want_fast != 0 it also prepares the hierarchical
 * evaluation (want_fast = 1 with its pyramid workspace; 2 without it, for
 * ndl_apply_fast_noalloc) (Section 3: the dyadic tree of panels; the per-node
 * decomposition of Step 1 is evaluated in closed form per panel row, so
 * nothing per node is stored).  This is the amortised set-up that the
 * paper's timings exclude. */
int ndl_plan_create(const ndl_problem* prob, int want_fast, ndl_plan* out, void* stream);
int ndl_plan_destroy(ndl_plan plan);

typedef struct {
    int64_t n_points;     /* n^dim */
    int64_t k_max, k_min; /* extreme integer cutoffs over the grid */
    int32_t ncomp;
    int32_t tile_x, tile_y, tile_z; /* tile of the direct kernel in use */
    int32_t variant;      /* internal id of the direct kernel */
    int32_t fast_levels;  /* tree levels used by the hierarchical path (0 = none) */
    double pairs_per_point; /* average lattice-ball size (neighbours per node) */
    int32_t pair_order;   /* summation order of the direct kernel in use: 0 = pairs
                             by increasing |z|^2, 1 = column by column (unrolled),
                             2 = column by column for run-time horizons (2D
                             diffusion with J > 7); variants with the same order
                             give bitwise identical results */
    int32_t fast_method;  /* method of ndl_apply_fast: 0 = dyadic panels (Steps 1-3
                             of Section 3), 1 = row prefix sums */
} ndl_plan_info;
int ndl_plan_get_info(ndl_plan plan, ndl_plan_info* info);

/* Direct quadrature sum (the "Original" operator of the paper's tables):
 * Lu = L u for `batch` states.  u and Lu as described above. */
int ndl_apply(ndl_plan plan, const void* u, void* Lu, int batch, void* stream);

/* Hierarchical evaluation of Section 3: Step 2 (bottom-up partial sums of u
 * over the dyadic panels) and Step 3 (sum over the panels of each node's
 * decomposition, combined by eq. "nonlocalP"), for the truncated polynomial
 * part p^0 = g(1); the remainder kappa = g - g(1) (zero for CONST) is summed
 * directly in the same pass.  Same inputs and result as ndl_apply up to
 * rounding.  Needs a plan made with want_fast != 0; case (a), diffusion. */
int ndl_apply_fast(ndl_plan plan, const void* u, void* Lu, int batch, void* stream);

/* ndl_apply_fast for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, with the pyramid of partial sums in a static
 * device workspace of 64 MiB that the library holds on each GPU it runs on
 * until the process ends, instead of the plan's own buffer.  The call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * the plan may be created with want_fast = 2, which skips the plan's pyramid
 * buffer.  Returns NDL_EINVAL when the plan's pyramid needs more than the
 * workspace holds (about n^dim / (2^dim - 1) doubles).  Every call on one GPU
 * shares that GPU's workspace and overwrites it before reading it, so calls
 * that overlap on one GPU (different streams, or threads without ordering)
 * race; calls ordered on one stream do not. */
int ndl_apply_fast_noalloc(ndl_plan plan, const void* u, void* Lu, int batch, void* stream);

/* Method of the hierarchical path of a plan made with want_fast != 0:
 * 0 = the dyadic panels of Section 3 (default); 1 = row prefix sums, the
 * variant with per-row interval sums in place of the dyadic decomposition
 * (the "other geometries than boxes" of the conclusion): Step 2 becomes
 * compensated FP64 prefix sums of u along every row of the padded box, and
 * Step 3 sums, per node, the 2J+1 (2D; (2J+1)^2 in 3D) row intervals of its
 * ball.  The row method serves diffusion with a degree-0 polynomial part
 * (power profiles and K = 0); NDL_EUNSUPPORTED otherwise.  ndl_autotune on
 * such a plan also times both methods and keeps the faster. */
int ndl_plan_set_fast_method(ndl_plan plan, int method);

/* Step 1 as used by ndl_apply_fast, for one node (test hook): writes up to cap
 * panels as (s, j_1..j_dim) int32 records, s = log2 of the panel side in
 * nodes and j the panel index on each axis of the tree over Omega, and sets
 * *count to the number of panels.  Host output buffer. */
int ndl_fast_decomposition(ndl_plan plan, const int64_t* node, int32_t* panels, int32_t cap,
                           int32_t* count);

/* The same Step 1 routine evaluated on the host, with no plan and no GPU:
 * the panels of the decomposition of the lattice ball {0 <= |z|^2 <= k} around
 * `node` (dim coordinates in [0, n)) cut by Omega, as records
 * (s, j_1..j_dim) like ndl_fast_decomposition. */
int ndl_decompose_node(int32_t dim, int64_t n, const int64_t* node, int64_t k, int32_t* panels,
                       int32_t cap, int32_t* count);

/* Batched CG on -L x = b (case (b), or the kernel-averaged form; zero volume
 * constraint), one independent problem per plan (uneven sizes allowed).
 * NDL_SYM plans (FP64) run Jacobi-CG one problem after another, with the
 * direct apply or, with opts->use_fast, the fast evaluation (the case (a)
 * hierarchical gather plus its adjoint scatter); the final residual is
 * recomputed with the direct apply.  For case (b):  b, x: device FP64 arrays of n^dim
 * (x holds the start value).  Stops when the FP64 true residual
 * ||b + L x|| / ||b|| <= rtol.  With NDL_F32C plans the inner iterations use
 * the compensated FP32 apply inside an FP64 iterative refinement; dot
 * products and norms are always FP64.  The inner iterations of all problems
 * run as one captured HIP graph of batched kernels; converged problems are
 * masked on the device. */
typedef struct {
    double rtol;          /* target relative residual (e.g. 1e-8) */
    int32_t max_iter;     /* cap on total inner iterations per problem */
    int32_t precond;      /* 0 = Jacobi, 1 = learned network (net must be set) */
    void* net;            /* ndl_net for precond == 1 */
    int32_t graph_iters;  /* iterations per captured graph launch (0 = default) */
    double inner_rtol;    /* refinement: inner reduction per outer step (0 = default) */
    int32_t use_fast;     /* NDL_SYM plans: iterate with ndl_apply_fast (plans made with want_fast) */
} ndl_cg_opts;

typedef struct {
    int32_t iters;        /* inner CG iterations */
    int32_t outer;        /* FP64 refinement steps */
    int32_t converged;    /* 1 if rel_res_fp64 <= rtol */
    int32_t fell_back;    /* 1 if the learned preconditioner was replaced by Jacobi */
    double rel_res_fp64;  /* final true residual */
    double seconds;       /* wall time of the whole batched solve */
} ndl_cg_report;

int ndl_cg_solve(const ndl_plan* plans, int nprob, const double* const* b, double* const* x,
                 const ndl_cg_opts* opts, ndl_cg_report* reports, void* stream);

/* Learned preconditioner: a 3D U-Net of 3x3x3 convolutions (BF16 weights
 * and activations, FP32 accumulation on MFMA), inputs (r / ||r||, standardised
 * log c, m / 4), output the correction z with z ~ (-L)^-1 r. */
typedef struct ndl_net_s* ndl_net;
int ndl_net_create(int levels, const int* channels, uint64_t seed, ndl_net* out);
int ndl_net_destroy(ndl_net net);
/* Linear mode of the preconditioner network (linear != 0): no activations and
 * no biases, the input is the residual alone, and residual and output are
 * scaled by D^-1/2 (D the diagonal of A = -L of the plan), so that
 * M(r) = D^-1/2 N(D^-1/2 r) is linear in r and sees delta and c through D.
 * Applies to inference, training and the learned PCG of an FP32 case (b)
 * plan; weights files are shared between modes. */
int ndl_net_set_linear(ndl_net net, int linear);
int ndl_net_save(ndl_net net, const char* path);
int ndl_net_load(ndl_net net, const char* path);
int ndl_net_num_params(ndl_net net, int64_t* count);
/* One Adam step on a minibatch of `batch` crops: r, e are device FP32 arrays
 * [batch][s^3] (residual and target correction), feat [batch][2][s^3] the
 * (log c, m/4) features; returns the mean loss in *loss. */
int ndl_net_train_step(ndl_net net, int batch, int s, const float* r, const float* feat,
                       const float* e, float lr, float* loss, void* stream);
/* One Adam step of energy-norm training on full fields of an FP32 3D case (b)
 * plan (n divisible by 8): for each of the `batch` samples (r, e) [batch][n^3]
 * (device FP32, A e = r with A = -L), the two-level preconditioner
 * z = D^-1 r + M(r) is evaluated and the loss ||e - z||_A^2 / ||e||_A^2 is
 * back-propagated; *loss is its batch mean. */
int ndl_net_train_step_energy(ndl_net net, ndl_plan plan, int batch, const float* r, const float* e, float lr,
                              float* loss, void* stream);
/* z = M(r), the network's part of the two-level preconditioner (the solver
 * adds D^-1 r): r, z device arrays of n^3 (element type of the plan's prec).
 * The plan (3D, n divisible by 8) supplies delta and c for the features; in
 * linear mode it must be an FP32 case (b) plan, whose -L diagonal D (built
 * once and cached with the plan's operator tables) scales the residual and
 * the output.  Guide for the solver, not a solve: its quality is measured by
 * ndl_cg_solve(precond = 1). */
int ndl_precond_apply(ndl_net net, ndl_plan plan, const void* r, void* z, void* stream);

/* Test hook: copy one FP32 tensor of network layer `layer` (0..12, in the
 * order input layer, encoder, bottom, decoder, output layer) to the host
 * buffer `out` of `count` values, which must equal the tensor's size.
 * which: 0 weights [cout][KP] (KP = 27 cin rounded up to 32, k = tap cin + c),
 * 1 biases [cout], 2 / 3 their gradients from the last training step,
 * 4 / 5 Adam's first and second moments of the weights, 6 / 7 those of the
 * biases.  Synchronises the device. */
int ndl_net_layer_tensor(ndl_net net, int layer, int which, float* out, int64_t count);

/* Test hook: one 3x3x3 convolution layer of the network (zero padding) with
 * the network's kernels.  x [S^3][cin] BF16 bit patterns (NDHWC), w
 * [cout][K] FP32 with K = 27 cin rounded up to 32 and k = tap cin + c,
 * tap = (dz*3 + dy)*3 + dx, bias [cout].  Outputs (each optional, NULL to
 * skip): y = conv(x) + bias, FP32 [S^3][cout] (weights and inputs rounded to
 * BF16, FP32 accumulation); dx = conv^T(dy), FP32 [S^3][cin] (dy rounded to
 * BF16); gw [cout][K], gb [cout] = weight and bias gradients for dy (FP32).
 * cin/cout in {(8,16), (16,16), (16,32), (32,32), (32,16)}.  Device pointers;
 * synchronises the stream. */
int ndl_net_conv_test(int cin, int cout, int S, const uint16_t* x, const float* w, const float* bias, float* y,
                      const float* dy, float* dx, float* gw, float* gb, void* stream);

/* Autotuner: time the candidate tiles of the direct kernel for this plan and
 * keep the fastest (cached in memory and in the file named by
 * NDL_AUTOTUNE_CACHE, if set).  Returns the chosen tile in the plan info. */
int ndl_autotune(ndl_plan plan, void* stream);

/* The same search on the caller's own state u (layout of ndl_apply) at the
 * caller's batch, timing applies of u into a scratch output; cached per
 * batch.  Use it when the plan serves batched calls (the best tile for one
 * field need not be the best for eight). */
int ndl_autotune_apply(ndl_plan plan, const void* u, int batch, void* stream);

/* The batched case (b) apply that ndl_cg_solve iterates: y_i = -L x_i with
 * the zero volume constraint for nprob case (b) diffusion plans (power
 * profile; one dimension, precision class and profile) in one persistent
 * launch over the tiles of all of them (Section 2, case (b)).  x_i, y_i:
 * device arrays of n_i^dim values of the plans' element type.  variant picks
 * the launch shape (nodes per lane and persistent grid size), 0 <= variant <
 * *nvariants, or -1 for the autotuner's choice for this batch (timed here on
 * x when not cached; ndl_cg_solve tunes the same way before it captures its
 * graph).  Every variant gives bitwise the same y.  variant_used and
 * nvariants (optional host pointers) report the variant run and the size of
 * the space (1 when the batch runs the generic kernel).  Allocates its
 * concatenated buffers; synchronises the stream. */
int ndl_div_batch_apply(const ndl_plan* plans, int nprob, const void* const* x, void* const* y, int variant,
                        int* variant_used, int* nvariants, void* stream);

/* Force a tile variant of the direct kernel (0 <= variant < ndl_plan_num_variants;
 * the autotuner's search space).  For tests and fixed deployments. */
int ndl_plan_set_variant(ndl_plan plan, int variant);
int ndl_plan_num_variants(ndl_plan plan, int* count);

const char* ndl_last_error(void);
const char* ndl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NDL_H */
