/*
 * Sanitizer run of the oracle (test infrastructure): its entry points on
 * small 1D, 2D and 3D problems, every profile and form, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.
 * On the way it checks the invariant that every form maps a constant state
 * (collar included) to zero, and that the decomposition of a node's ball
 * counts the ball's lattice points inside Omega.  Exit status 0 on success.
 */
#include "../oracle/ndl_oracle.c"

#include <stdio.h>

static double frand(uint64_t* s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

static int run_case(int dim, int64_t n, int model, int form, int kernel, uint64_t seed)
{
    static const double poly[3] = {1.0, -0.5, 0.1};
    or_problem p;
    memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.n = n;
    p.R = 4;
    p.model = model;
    p.form = form;
    p.kernel = kernel;
    p.s = 0.5;
    p.K = kernel == 3 ? 2 : 0;
    p.poly = poly;
    p.norm = 0;
    p.m2 = model ? 2.0 * dim * (dim + 2) : 2.0 * dim;
    const int nc = model ? dim : 1;
    const int64_t N = ipow(n, dim), P = ipow(n + 2 * p.R, dim);
    double* delta = malloc(N * sizeof(double));
    double* coef = malloc(N * sizeof(double));
    double* u = malloc(nc * P * sizeof(double));
    double* out = malloc(nc * N * sizeof(double));
    for (int64_t i = 0; i < N; i++) {
        delta[i] = (1.0 + 1.5 * frand(&seed)) / (double)n; /* m in [1, 2.5] */
        coef[i] = 0.5 + 1.5 * frand(&seed);
    }
    int bad = 0;
    for (int pass = 0; pass < 2; pass++) {
        /* pass 0: a constant state, pass 1: a random one */
        for (int64_t i = 0; i < nc * P; i++) u[i] = pass == 0 ? 1.25 : frand(&seed) - 0.5;
        int rc = form == 0 ? or_apply_nd(&p, delta, coef, u, out)
               : form == 1 ? or_apply_div(&p, delta, coef, u, out)
                           : or_apply_sym(&p, delta, coef, u, out);
        if (rc != 0) {
            fprintf(stderr, "apply failed: dim %d model %d form %d kernel %d\n", dim, model, form, kernel);
            bad = 1;
            break;
        }
        double mx = 0.0;
        for (int64_t i = 0; i < nc * N; i++) mx = fmax(mx, fabs(out[i]));
        if (pass == 0 && !(mx <= 1e-9)) {
            fprintf(stderr, "L const = %g: dim %d model %d form %d kernel %d\n", mx, dim, model, form, kernel);
            bad = 1;
        }
        if (pass == 1 && !isfinite(mx)) bad = 1;
    }
    if (form == 1 && model == 0) {
        double* diag = malloc(N * sizeof(double));
        if (or_div_diag(&p, delta, coef, diag) != 0) bad = 1;
        free(diag);
    }
    free(delta);
    free(coef);
    free(u);
    free(out);
    return bad;
}

static int run_decompose(int dim, int64_t n, int64_t k)
{
    int64_t cap = 4096;
    int* lev = malloc(cap * sizeof(int));
    int64_t* idx = malloc(cap * 3 * sizeof(int64_t));
    int bad = 0;
    int64_t c[3] = {0, 0, 0};
    for (int64_t t = 0; t < ipow(n, dim); t += 3) {
        int64_t r = t;
        for (int a = dim - 1; a >= 0; a--) { c[a] = r % n; r /= n; }
        int64_t cnt = or_decompose(dim, n, c, k, lev, idx, cap);
        if (cnt < 0 || cnt > cap) { bad = 1; break; }
        /* the panels' node counts add up to the ball's lattice points in Omega */
        int L = or_tree_levels(n);
        int64_t nodes = 0;
        for (int64_t q = 0; q < cnt; q++) {
            int64_t side = (int64_t)1 << (L - lev[q]);
            int64_t in = 1;
            for (int a = 0; a < dim; a++) {
                int64_t lo = idx[q * dim + a] * side, hi = lo + side;
                if (hi > n) hi = n;
                in *= hi > lo ? hi - lo : 0;
            }
            nodes += in;
        }
        int64_t want = 0, z[3] = {0, 0, 0}, J = (int64_t)sqrt((double)k) + 1;
        int64_t lo1 = dim >= 2 ? -J : 0, hi1 = dim >= 2 ? J : 0, lo2 = dim >= 3 ? -J : 0, hi2 = dim >= 3 ? J : 0;
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                    if (z[0] * z[0] + z[1] * z[1] + z[2] * z[2] > k) continue;
                    int ok = 1;
                    for (int a = 0; a < dim; a++)
                        if (c[a] + z[a] < 0 || c[a] + z[a] >= n) ok = 0;
                    want += ok;
                }
        if (nodes != want) {
            fprintf(stderr, "decomposition of node %lld: %lld nodes, ball %lld\n", (long long)t, (long long)nodes,
                    (long long)want);
            bad = 1;
            break;
        }
    }
    free(lev);
    free(idx);
    return bad;
}

int main(void)
{
    int bad = 0, cases = 0;
    const int64_t ns[4] = {0, 11, 7, 5};
    for (int dim = 1; dim <= 3; dim++)
        for (int model = 0; model <= (dim >= 2 ? 1 : 0); model++)
            for (int form = 0; form <= 2; form++)
                for (int kernel = 0; kernel <= 4; kernel++) {
                    if (model == 1 && form != 0) continue;
                    bad |= run_case(dim, ns[dim], model, form, kernel, 1000u + 97u * (unsigned)(dim * 100 + model * 10 + form) + (unsigned)kernel);
                    cases++;
                }
    for (int dim = 1; dim <= 3; dim++) bad |= run_decompose(dim, ns[dim] + 2, dim == 1 ? 9 : 5);
    printf("%d apply cases, decompositions in 1D/2D/3D: %s\n", cases, bad ? "FAILED" : "ok");
    return bad;
}
