// The extern "C" entry points of include/ndl.h: argument checking, plan
// lifetime, dispatch to the kernels, thread-local error messages.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "common.h"

namespace ndl {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char* what, const char* file, int line)
{
    set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
    return e == hipErrorOutOfMemory ? NDL_ENOMEM : NDL_EHIP;
}

static void free_plan(Plan* p)
{
    if (!p) return;
    void* bufs[] = {p->d_k, p->d_scale, p->d_invm2, p->d_split, p->d_invT, p->d_pairs, p->d_pairw, p->d_wq,
                    p->d_full, p->d_fullw, p->d_pyr, p->d_wtab, p->d_symws, p->d_kseg};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int32_t* b : p->d_tord)
        if (b) (void)hipFree(b);
    delete p;
}

static int validate(const ndl_problem* q)
{
    if (!q) { set_error("null problem"); return NDL_EINVAL; }
    if (q->dim < 1 || q->dim > 3) { set_error("dim must be 1, 2 or 3 (got %d)", q->dim); return NDL_EINVAL; }
    if (q->n < 1) { set_error("n must be >= 1"); return NDL_EINVAL; }
    int64_t P = q->n + 2 * (int64_t)q->collar;
    double tot = std::pow((double)P, q->dim);
    if (q->collar < 0 || tot > 4.0e9) { set_error("collar/grid out of range"); return NDL_EINVAL; }
    if (q->model != NDL_DIFFUSION && q->model != NDL_PERIDYNAMIC) { set_error("bad model"); return NDL_EINVAL; }
    if (q->model == NDL_PERIDYNAMIC && q->dim < 2) {
        set_error("peridynamic model is implemented for dim 2 and 3");
        return NDL_EUNSUPPORTED;
    }
    if (q->form != NDL_ND && q->form != NDL_DIV && q->form != NDL_SYM) { set_error("bad form"); return NDL_EINVAL; }
    if (q->form == NDL_SYM && (q->model != NDL_DIFFUSION || q->kernel > NDL_G_FRAC)) {
        set_error("the kernel-averaged form is implemented for diffusion with a power profile");
        return NDL_EUNSUPPORTED;
    }
    if (q->form == NDL_DIV && q->model == NDL_PERIDYNAMIC) {
        set_error("case (b) is implemented for the diffusion model");
        return NDL_EUNSUPPORTED;
    }
    if (q->kernel < 0 || q->kernel > NDL_G_CONE) { set_error("bad kernel"); return NDL_EINVAL; }
    if (q->kernel == NDL_G_CONE && q->form == NDL_DIV) {
        set_error("case (b) supports the power profiles only");
        return NDL_EUNSUPPORTED;
    }
    if (q->kernel == NDL_G_FRAC && !(q->s >= 0.0 && q->s < 1.0)) {
        set_error("fractional order s must be in [0, 1)");
        return NDL_EINVAL;
    }
    if (q->kernel == NDL_G_POLY) {
        if (!q->poly || q->K < 0 || q->K > 7) { set_error("POLY needs 0 <= K <= 7 and K+1 coefficients"); return NDL_EINVAL; }
        if (q->form == NDL_DIV) { set_error("case (b) supports the power profiles only"); return NDL_EUNSUPPORTED; }
    }
    if (q->norm < 0 || q->norm > NDL_NORM_NONE) { set_error("bad norm"); return NDL_EINVAL; }
    if (q->prec != NDL_F64 && q->prec != NDL_F32C && q->prec != NDL_F32K) { set_error("bad prec"); return NDL_EINVAL; }
    if (!q->delta || !q->coef) { set_error("delta and coef must be device pointers"); return NDL_EINVAL; }
    return NDL_OK;
}

}  // namespace ndl

using namespace ndl;

extern "C" {

const char* ndl_last_error(void) { return g_err; }
const char* ndl_version(void) { return "ndl 0.1 (gfx950)"; }

int ndl_plan_create(const ndl_problem* prob, int want_fast, ndl_plan* out, void* stream)
{
    if (!out) { set_error("null output handle"); return NDL_EINVAL; }
    *out = nullptr;
    NDL_TRY(validate(prob));
    Plan* p = new (std::nothrow) Plan();
    if (!p) { set_error("host allocation failed"); return NDL_ENOMEM; }
    p->prob = *prob;
    if (prob->kernel == NDL_G_POLY) p->poly.assign(prob->poly, prob->poly + prob->K + 1);
    p->prob.poly = p->poly.empty() ? nullptr : p->poly.data();
    p->dim = prob->dim;
    p->n = prob->n;
    p->R = prob->collar;
    p->model = prob->model;
    p->form = prob->form;
    p->kernel = prob->kernel;
    p->norm = prob->norm;
    p->prec = prob->prec;
    p->ncomp = prob->model == NDL_PERIDYNAMIC ? prob->dim : 1;
    p->N = 1;
    p->NP = 1;
    p->P = p->n + 2 * p->R;
    for (int a = 0; a < p->dim; a++) { p->N *= p->n; p->NP *= p->P; }
    p->m2 = prob->m2_target > 0 ? prob->m2_target
                                : (p->model == NDL_PERIDYNAMIC ? 2.0 * p->dim * (p->dim + 2) : 2.0 * p->dim);
    switch (p->kernel) {
    case NDL_G_CONST: p->expo = 0.0; break;
    case NDL_G_INV_R: p->expo = -1.0; break;
    case NDL_G_FRAC: p->expo = -((double)p->dim + 2.0 * prob->s); break;
    case NDL_G_CONE: p->expo = -1.0; break;  // the 1/r factor (weights formed per pair)
    default: p->expo = 0.0; break;
    }
    hipStream_t s = (hipStream_t)stream;
    int rc = plan_fields(*p, s);
    if (rc == NDL_OK) rc = tile_orders_2d(*p, s);
    if (rc == NDL_OK && want_fast) {
        rc = fast_prepare(*p, s, want_fast != 2);
        if (rc == NDL_OK && p->form == NDL_SYM) {
            if (want_fast == 2) {
                set_error("the kernel-averaged form's fast evaluation needs its workspace (want_fast = 1)");
                rc = NDL_EUNSUPPORTED;
            } else {
                rc = sym_prepare(*p, s);
            }
        }
    }
    if (rc != NDL_OK) { free_plan(p); return rc; }
    *out = reinterpret_cast<ndl_plan>(p);
    return NDL_OK;
}

int ndl_plan_destroy(ndl_plan plan)
{
    free_plan(reinterpret_cast<Plan*>(plan));
    return NDL_OK;
}

int ndl_plan_get_info(ndl_plan plan, ndl_plan_info* info)
{
    if (!plan || !info) { set_error("null argument"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    memset(info, 0, sizeof(*info));
    info->n_points = p->N;
    info->k_max = p->kmax;
    info->k_min = p->kmin;
    info->ncomp = p->ncomp;
    info->tile_x = p->tile_x;
    info->tile_y = p->tile_y;
    info->tile_z = p->tile_z;
    if (direct_2d_applies(*p)) {
        variant_tile_2d(*p, p->variant, &info->tile_x, &info->tile_y);
        info->tile_z = 1;
        info->pair_order = variant_order_2d(*p, p->variant);
    }
    info->variant = p->variant;
    info->fast_levels = p->fast ? p->fast_S + 1 : 0;
    info->pairs_per_point = p->avg_ball;
    info->fast_method = p->fast_method;
    return NDL_OK;
}

int ndl_plan_set_fast_method(ndl_plan plan, int method)
{
    if (!plan) { set_error("null plan"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p->fast) { set_error("plan was created without want_fast"); return NDL_EINVAL; }
    if (method < 0 || method > 1) { set_error("fast method %d: 0 (dyadic panels) or 1 (row prefix sums)", method); return NDL_EINVAL; }
    if (method >= fast_num_methods(*p)) {
        set_error("the row method serves diffusion with a degree-0 polynomial part");
        return NDL_EUNSUPPORTED;
    }
    p->fast_method = method;
    return NDL_OK;
}

int ndl_apply(ndl_plan plan, const void* u, void* Lu, int batch, void* stream)
{
    if (!plan || !u || !Lu || batch < 0) { set_error("ndl_apply: null argument or negative batch"); return NDL_EINVAL; }
    if (batch == 0 || reinterpret_cast<Plan*>(plan)->N == 0) return NDL_OK;
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (batch > 65535) { set_error("batch too large (max 65535)"); return NDL_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (p->form == NDL_DIV) return launch_div(*p, u, Lu, batch, s);
    if (p->form == NDL_SYM) return launch_sym(*p, u, Lu, batch, s);
    return launch_direct(*p, u, Lu, batch, s);
}

int ndl_apply_fast(ndl_plan plan, const void* u, void* Lu, int batch, void* stream)
{
    if (!plan || !u || !Lu || batch < 0) { set_error("ndl_apply_fast: null argument"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p->fast) { set_error("plan was created without want_fast"); return NDL_EINVAL; }
    if (!p->d_pyr) {
        set_error("plan was created without its pyramid workspace (want_fast = 2): use ndl_apply_fast_noalloc");
        return NDL_EINVAL;
    }
    if (batch == 0) return NDL_OK;
    if (p->form == NDL_SYM) return launch_sym_fast(*p, u, Lu, batch, (hipStream_t)stream);
    return launch_fast(*p, u, Lu, batch, (hipStream_t)stream);
}

int ndl_apply_fast_noalloc(ndl_plan plan, const void* u, void* Lu, int batch, void* stream)
{
    if (!plan || !u || !Lu || batch < 0) { set_error("ndl_apply_fast_noalloc: null argument"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p->fast) { set_error("plan was created without want_fast"); return NDL_EINVAL; }
    double* ws = nullptr;
    int64_t cap = 0;
    NDL_TRY(fast_static_workspace(&ws, &cap));
    if (p->form == NDL_SYM) {
        set_error("ndl_apply_fast_noalloc: the kernel-averaged form keeps a plan workspace (use ndl_apply_fast)");
        return NDL_EUNSUPPORTED;
    }
    if (p->pyr_elems > cap) {
        set_error("ndl_apply_fast_noalloc: the pyramid needs %lld bytes, the static workspace holds %lld",
                  (long long)(p->pyr_elems * (int64_t)sizeof(double)), (long long)(cap * (int64_t)sizeof(double)));
        return NDL_EINVAL;
    }
    if (batch == 0) return NDL_OK;
    return launch_fast(*p, u, Lu, batch, (hipStream_t)stream, ws);
}

int ndl_fast_decomposition(ndl_plan plan, const int64_t* node, int32_t* panels, int32_t cap, int32_t* count)
{
    if (!plan || !node || !count || (cap > 0 && !panels)) { set_error("null argument"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p->fast) { set_error("plan was created without want_fast"); return NDL_EINVAL; }
    int c = 0;
    int rc = fast_decomp_host(*p, node, panels, cap, &c);
    *count = c;
    return rc;
}

int ndl_plan_num_variants(ndl_plan plan, int* count)
{
    if (!plan || !count) { set_error("null argument"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    *count = direct_2d_applies(*p) ? num_variants_2d() : 1;
    return NDL_OK;
}

int ndl_plan_set_variant(ndl_plan plan, int variant)
{
    if (!plan) { set_error("null plan"); return NDL_EINVAL; }
    Plan* p = reinterpret_cast<Plan*>(plan);
    int nv = direct_2d_applies(*p) ? num_variants_2d() : 1;
    if (variant < 0 || variant >= nv) { set_error("variant %d out of range [0, %d)", variant, nv); return NDL_EINVAL; }
    p->variant = variant;
    return NDL_OK;
}

int ndl_autotune(ndl_plan plan, void* stream)
{
    if (!plan) { set_error("null plan"); return NDL_EINVAL; }
    return autotune(*reinterpret_cast<Plan*>(plan), (hipStream_t)stream);
}

int ndl_autotune_apply(ndl_plan plan, const void* u, int batch, void* stream)
{
    if (!plan || !u || batch < 1 || batch > 65535) { set_error("ndl_autotune_apply: bad arguments"); return NDL_EINVAL; }
    return autotune_apply(*reinterpret_cast<Plan*>(plan), u, batch, (hipStream_t)stream);
}

}  // extern "C"
