// Tile autotuner for the direct kernels: times every tile variant of the
// kernel a plan uses (hipEvents, on the caller's stream) and keeps the
// fastest: either on a scratch state of ones at batch 1 (ndl_autotune) or on
// the caller's own state at the caller's batch (ndl_autotune_apply).  Results
// are cached per (dim, form, model, prec, reach J, n, ncomp, profile, batch)
// in memory and, when NDL_AUTOTUNE_CACHE names a file, in that file ("key
// variant" lines) so later processes skip the search.  The batched case (b)
// solver keeps its launch variants in the same cache.
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <vector>
#include <sstream>
#include <string>

#include "common.h"

namespace ndl {

static std::mutex g_mu;
static std::map<std::string, int> g_cache;
static bool g_loaded = false;

static std::string key_of(const Plan& p, int batch)
{
    std::ostringstream k;
    k << "d" << p.dim << ".f" << p.form << ".m" << p.model << ".p" << p.prec << ".J" << p.J << ".n" << p.n
      << ".c" << p.ncomp << ".g" << p.kernel << ".b" << batch;
    return k.str();
}

static void load_file()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* fn = std::getenv("NDL_AUTOTUNE_CACHE");
    if (!fn) return;
    std::ifstream f(fn);
    std::string k;
    int v;
    while (f >> k >> v) g_cache[k] = v;
}

static void save_file(const std::string& k, int v)
{
    const char* fn = std::getenv("NDL_AUTOTUNE_CACHE");
    if (!fn) return;
    std::ofstream f(fn, std::ios::app);
    f << k << " " << v << "\n";
}

bool tune_cache_lookup(const std::string& key, int* variant)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_file();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *variant = it->second;
    return true;
}

void tune_cache_store(const std::string& key, int variant)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = variant;
    save_file(key, variant);
}



// time every variant applying L to u (batch states) into out; keep the fastest
static int tune_variants(Plan& p, const void* u, void* out, int batch, hipStream_t s, int* best_out)
{
    hipEvent_t e0, e1;
    NDL_HIP(hipEventCreate(&e0));
    NDL_HIP(hipEventCreate(&e1));
    // three rounds over all variants (timed launches after warm ones); a
    // variant's time is its best round, which keeps clock ramps and
    // neighbours' noise out of the comparison of near-equal tiles
    const int nv = num_variants_2d();
    const int reps = std::max(2, 20 / std::max(1, batch));
    std::vector<float> t(nv, 1e30f);
    int rc = NDL_OK;
    for (int round = 0; round < 3 && rc == NDL_OK; ++round) {
        for (int v = 0; v < nv && rc == NDL_OK; ++v) {
            p.variant = v;
            for (int w = 0; w < 2 && rc == NDL_OK; ++w) rc = launch_direct(p, u, out, batch, s);
            if (rc != NDL_OK) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == NDL_OK; ++r) rc = launch_direct(p, u, out, batch, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t[v] = std::min(t[v], ms);
        }
    }
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (t[v] < t[best]) best = v;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_out = best;
    return rc;
}

__global__ void k_fill_ones(float* a, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 1.0f;
}

// the faster method of the hierarchical path (dyadic panels or row prefix sums)
static int autotune_fast(Plan& p, hipStream_t s)
{
    if (fast_num_methods(p) < 2 || !p.d_pyr) return NDL_OK;
    const std::string key = "fast." + key_of(p, 1);
    int cached = 0;
    if (tune_cache_lookup(key, &cached)) {
        p.fast_method = cached;
        return NDL_OK;
    }
    size_t es = elem_size(p.prec);
    void *u = nullptr, *o = nullptr;
    NDL_HIP(hipMalloc(&u, (size_t)p.NP * es));
    NDL_HIP(hipMalloc(&o, (size_t)p.N * es));
    const int64_t nf = (int64_t)(p.NP * es / sizeof(float));
    k_fill_ones<<<(unsigned)((nf + 255) / 256), 256, 0, s>>>((float*)u, nf);
    hipEvent_t e0, e1;
    NDL_HIP(hipEventCreate(&e0));
    NDL_HIP(hipEventCreate(&e1));
    float t[2] = {1e30f, 1e30f};
    int rc = NDL_OK;
    for (int round = 0; round < 3 && rc == NDL_OK; ++round)
        for (int m = 0; m < 2 && rc == NDL_OK; ++m) {
            p.fast_method = m;
            rc = launch_fast(p, u, o, 1, s);
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 5 && rc == NDL_OK; ++r) rc = launch_fast(p, u, o, 1, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t[m] = std::min(t[m], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(u);
    (void)hipFree(o);
    p.fast_method = t[1] < t[0] ? 1 : 0;
    if (rc != NDL_OK) return rc;
    tune_cache_store(key, p.fast_method);
    return NDL_OK;
}

int autotune(Plan& p, hipStream_t s)
{
    NDL_TRY(autotune_fast(p, s));
    if (!direct_2d_applies(p)) return NDL_OK;  // one variant only
    const std::string key = key_of(p, 1);
    int cached = 0;
    if (tune_cache_lookup(key, &cached)) {
        p.variant = cached;
        return NDL_OK;
    }
    size_t es = elem_size(p.prec);
    void *u = nullptr, *o = nullptr;
    NDL_HIP(hipMalloc(&u, (size_t)p.NP * p.ncomp * es));
    NDL_HIP(hipMalloc(&o, (size_t)p.N * p.ncomp * es));
    // a state of ones (any non-zero data; the kernels' work does not depend on it)
    const int64_t nf = (int64_t)(p.NP * p.ncomp * es / sizeof(float));
    k_fill_ones<<<(unsigned)((nf + 255) / 256), 256, 0, s>>>((float*)u, nf);
    int best = 0;
    int rc = tune_variants(p, u, o, 1, s, &best);
    (void)hipFree(u);
    (void)hipFree(o);
    p.variant = best;
    if (rc != NDL_OK) return rc;
    tune_cache_store(key, best);
    return NDL_OK;
}

int autotune_apply(Plan& p, const void* u, int batch, hipStream_t s)
{
    if (!direct_2d_applies(p)) return NDL_OK;
    const std::string key = key_of(p, batch);
    int cached = 0;
    if (tune_cache_lookup(key, &cached)) {
        p.variant = cached;
        return NDL_OK;
    }
    void* o = nullptr;
    NDL_HIP(hipMalloc(&o, (size_t)p.N * p.ncomp * batch * elem_size(p.prec)));
    int best = 0;
    int rc = tune_variants(p, u, o, batch, s, &best);
    (void)hipFree(o);
    p.variant = best;
    if (rc != NDL_OK) return rc;
    tune_cache_store(key, best);
    return NDL_OK;
}

}  // namespace ndl
