/*
 * ndl_oracle.c -- plain, slow, FP64 CPU oracle for the nonlocal operators of
 * Tian & Engquist, "Fast algorithm for computing nonlocal operators with finite
 * interaction distance" (arXiv 1905.08375).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the GPU library; the two never include or link each
 * other.
 *
 * Everything is written straight from the definitions, in FP64, with no
 * blocking, fusion or reordering.  Compile with -ffp-contract=off so that no
 * multiply-add is fused.  OpenMP only splits the outer loop over grid nodes.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - grid: Omega = [0,1]^d, n nodes per axis, h = 1/n, node i sits at (i+1/2)h;
 *  - state u is given on the padded index box {-R..n-1+R}^d; the collar holds
 *    the volume-constraint data (zero for the homogeneous Dirichlet problem of
 *    Section 3, problem "nonlocal:polynomial");
 *  - the horizon ball is strict, |y-x| < delta (kernel profile support, eq.
 *    "kernelgamma"), taken on the lattice as 0 < |z|^2 <= k with
 *    k = ceil((delta*n)*(delta*n)) - 1 evaluated in IEEE FP64 in that order;
 *  - the kernel is omega(x,y) = C * A * g(|y-x|/delta) (Section 2, eq. "kernel",
 *    with the normalising constant A made explicit, see or_norm below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim;            /* 1, 2 or 3 */
    int64_t n;          /* nodes per axis */
    int R;              /* collar width of the padded state */
    int model;          /* 0: scalar diffusion, 1: linear bond-based peridynamics (dim 2 or 3) */
    int form;           /* 0: case (a), C and delta depend on x only; 1: case (b), symmetrised;
                           2: kernel-averaged, omega_s(x,y) = (omega_x(y) + omega_y(x)) / 2 */
    int kernel;         /* profile g: 0 const, 1 1/r, 2 r^-(d+2s), 3 even polynomial p(r), 4 cone (1-r)/r */
    double s;           /* fractional order for kernel 2 */
    int K;              /* kernel 3: p(r) = sum_{j<=K} poly[j] r^(2j) */
    const double* poly;
    int norm;           /* 0 discrete second moment, 1 continuous second moment, 2 none */
    double m2;          /* second-moment target M (2d for diffusion, 2d(d+2) for PD) */
} or_problem;

/* ------------------------------------------------------------------ cutoff */
/* Lattice horizon: z belongs to the ball iff 0 < |z|^2 <= k (strict |y-x| < delta). */
int64_t or_cutoff(double delta, int64_t n)
{
    double a = delta * (double)n;
    double t = a * a;
    return (int64_t)ceil(t) - 1;
}

/* Case (b): the symmetric horizon delta_ij = (delta_i + delta_j)/2. */
int64_t or_cutoff_pair(double di, double dj, int64_t n)
{
    double a = (di + dj) * (double)n * 0.5;
    double t = a * a;
    return (int64_t)ceil(t) - 1;
}

static int64_t isqrt_floor(int64_t k)
{
    int64_t J = 0;
    while ((J + 1) * (J + 1) <= k) J++;
    return J;
}

/* ------------------------------------------------------------------ profile */
/* Radial profiles g(r), r = |y-x|/delta (Section 2: eq. "kernelgamma" gives 1/r
 * and the conical (1-r)/r, both on r < 1; the fractional type r^-(d+2s) is the
 * micromodulus family of Section 1; the even polynomial p^{2K} is the truncated
 * part of the splitting in Section 3). */
double or_profile(const or_problem* p, double r)
{
    switch (p->kernel) {
    case 0: return 1.0;
    case 1: return 1.0 / r;
    case 2: return pow(r, -((double)p->dim + 2.0 * p->s));
    case 3: {
        double r2 = r * r, pw = 1.0, acc = 0.0;
        for (int j = 0; j <= p->K; j++) { acc += p->poly[j] * pw; pw *= r2; }
        return acc;
    }
    case 4: return (1.0 - r) / r;
    }
    return 0.0;
}

/* |S^{d-1}|: length/area of the unit sphere in R^d. */
static double sphere_area(int d)
{
    if (d == 1) return 2.0;
    if (d == 2) return 2.0 * M_PI;
    return 4.0 * M_PI;
}

/* int_0^1 g(r) r^(d+1) dr in closed form. */
static double radial_moment(const or_problem* p)
{
    int d = p->dim;
    switch (p->kernel) {
    case 0: return 1.0 / (d + 2.0);
    case 1: return 1.0 / (d + 1.0);
    case 2: return 1.0 / (2.0 - 2.0 * p->s);
    case 3: {
        double acc = 0.0;
        for (int j = 0; j <= p->K; j++) acc += p->poly[j] / (2.0 * j + d + 2.0);
        return acc;
    }
    case 4: return 1.0 / (d + 1.0) - 1.0 / (d + 2.0); /* int_0^1 (1-r) r^d dr */
    }
    return 0.0;
}

/* Normalising constant A, so that omega(z) = C * A * g(|z|/m) and
 *   L u_i = sum_z omega(z) (u_{i+z} - u_i) h^d.
 * norm 0 (discrete):   A * sum_{0<|z|^2<=k} g(|z|/m) |z h|^2 h^d = M, so the
 *                      operator reproduces 2d (diffusion) on |x|^2 exactly;
 * norm 1 (continuous): A * int_{B_delta} g(|y|/delta) |y|^2 dy = M;
 * norm 2 (none):       A = delta^-(d+2), the literal constant of eq. "kernel". */
/* Exponent e of a power profile g(r) = r^e (kernels 0, 1, 2). */
static double power_exponent(const or_problem* p)
{
    if (p->kernel == 0) return 0.0;
    if (p->kernel == 1) return -1.0;
    return -((double)p->dim + 2.0 * p->s);
}

/* Memo of the lattice moment sums T_e[k] = sum_{0<|z|^2<=k} |z|^(e+2) for the
 * power profiles, where g(|z|/m) |z|^2 = m^-e |z|^(e+2) factors the
 * m-dependence out of the discrete normalisation sum.  Filled by enumeration. */
typedef struct {
    int64_t kmax;
    double* T;
} moment_memo;

static void memo_build(const or_problem* p, int64_t kmax, moment_memo* mm)
{
    int d = p->dim;
    double e = power_exponent(p);
    mm->kmax = kmax;
    mm->T = (double*)calloc((size_t)(kmax + 1), sizeof(double));
    int64_t J = isqrt_floor(kmax);
    int64_t z[3] = {0, 0, 0};
    int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
    int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
    for (z[0] = -J; z[0] <= J; z[0]++)
        for (z[1] = lo1; z[1] <= hi1; z[1]++)
            for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                if (q == 0 || q > kmax) continue;
                mm->T[q] += pow(sqrt((double)q), e + 2.0);
            }
    for (int64_t k = 1; k <= kmax; k++) mm->T[k] += mm->T[k - 1];
}

static const moment_memo* g_memo = NULL; /* set for the duration of one apply */

double or_norm(const or_problem* p, int64_t k, double m, double delta)
{
    int d = p->dim;
    double h = 1.0 / (double)p->n;
    if (p->norm == 2) return 1.0 / pow(delta, d + 2.0);
    if (p->norm == 1)
        return p->m2 / (sphere_area(d) * pow(delta, d + 2.0) * radial_moment(p));
    if (g_memo && p->kernel <= 2 && k <= g_memo->kmax) {
        double e = power_exponent(p);
        double T = g_memo->T[k];
        return T > 0.0 ? p->m2 * pow(m, e) / (pow(h, (double)d + 2.0) * T) : INFINITY;
    }
    double hd = pow(h, (double)d);
    int64_t J = isqrt_floor(k);
    double sum = 0.0;
    int64_t z[3] = {0, 0, 0};
    int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
    int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
    for (z[0] = -J; z[0] <= J; z[0]++)
        for (z[1] = lo1; z[1] <= hi1; z[1]++)
            for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                if (q == 0 || q > k) continue;
                double len = sqrt((double)q);
                sum += or_profile(p, len / m) * (len * h) * (len * h) * hd;
            }
    return p->m2 / sum;
}

/* ------------------------------------------------------------------ indexing */
static int64_t pidx(const or_problem* p, const int64_t* x) /* padded index of node x */
{
    int64_t P = p->n + 2 * p->R, off = 0;
    for (int a = 0; a < p->dim; a++) off = off * P + (x[a] + p->R);
    return off;
}

static int64_t gidx(const or_problem* p, const int64_t* x) /* grid index, x in Omega */
{
    int64_t off = 0;
    for (int a = 0; a < p->dim; a++) off = off * p->n + x[a];
    return off;
}

static void unflatten(const or_problem* p, int64_t i, int64_t* x)
{
    x[0] = x[1] = x[2] = 0;
    for (int a = p->dim - 1; a >= 0; a--) { x[a] = i % p->n; i /= p->n; }
}

static int in_omega(const or_problem* p, const int64_t* x)
{
    for (int a = 0; a < p->dim; a++)
        if (x[a] < 0 || x[a] >= p->n) return 0;
    return 1;
}

static int64_t npoints(const or_problem* p)
{
    int64_t N = 1;
    for (int a = 0; a < p->dim; a++) N *= p->n;
    return N;
}

/* ------------------------------------------------------------------ apply */
/* Case (a), eq. "eq:diffusion" with C = C(x), delta = delta(x):
 *   L u_i = sum_{0<|z|^2<=k_i} c_i A_i g(|z|/m_i) (u_{i+z} - u_i) h^d.
 * Peridynamics (Section 1, linear bond force), ncomp = d displacement components:
 *   L u_i = sum_z c_i A_i g(|z|/m_i) [e.(u_{i+z} - u_i)] e h^d,  e = z/|z|.
 * u: [ncomp][padded box], out: [ncomp][n^d].  Returns 0, or -1 if the collar
 * is narrower than the widest horizon. */
int or_apply_nd(const or_problem* p, const double* delta, const double* coef,
                const double* u, double* out)
{
    int d = p->dim;
    int64_t N = npoints(p);
    int64_t Pn = 1;
    for (int a = 0; a < d; a++) Pn *= (p->n + 2 * p->R);
    double h = 1.0 / (double)p->n;
    double hd = pow(h, (double)d);
    for (int64_t i = 0; i < N; i++)
        if (isqrt_floor(or_cutoff(delta[i], p->n)) > p->R) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        int64_t x[3], y[3], z[3] = {0, 0, 0};
        unflatten(p, i, x);
        double m = delta[i] * (double)p->n;
        int64_t k = or_cutoff(delta[i], p->n);
        double A = or_norm(p, k, m, delta[i]);
        int64_t J = isqrt_floor(k);
        int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
        int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
        double acc[3] = {0.0, 0.0, 0.0};
        int64_t xi = pidx(p, x);
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                    int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                    if (q == 0 || q > k) continue;
                    for (int a = 0; a < 3; a++) y[a] = x[a] + z[a];
                    int64_t yi = pidx(p, y);
                    double len = sqrt((double)q);
                    double w = coef[i] * A * or_profile(p, len / m);
                    if (p->model == 0) {
                        acc[0] += w * (u[yi] - u[xi]) * hd;
                    } else {
                        /* bond direction e and the projection e.(u(y) - u(x)) */
                        double e[3], proj = 0.0;
                        for (int c = 0; c < d; c++) {
                            e[c] = (double)z[c] / len;
                            proj += e[c] * (u[c * Pn + yi] - u[c * Pn + xi]);
                        }
                        for (int c = 0; c < d; c++) acc[c] += w * proj * e[c] * hd;
                    }
                }
        int nc = p->model == 1 ? d : 1;
        for (int c = 0; c < nc; c++) out[c * N + i] = acc[c];
    }
    return 0;
}

/* Case (b), eq. "eq:diffusion" with symmetric C and delta:
 *   C_ij = (c_i + c_j)/2, delta_ij = (delta_i + delta_j)/2, k_ij from delta_ij,
 *   L u_i = sum_{0<|z|^2<=k_ij} C_ij A(k_ij, m_ij) g(|z|/m_ij) (u_j - u_i) h^d,
 * where a partner j in the collar takes (delta_i, c_i). */
static double div_weight(const or_problem* p, const double* delta, const double* coef,
                         int64_t i, const int64_t* y, const int64_t* z, int64_t* kout)
{
    double dj = delta[i], cj = coef[i];
    if (in_omega(p, y)) { int64_t j = gidx(p, y); dj = delta[j]; cj = coef[j]; }
    int64_t kij = or_cutoff_pair(delta[i], dj, p->n);
    *kout = kij;
    int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
    if (q > kij) return 0.0;
    double dij = (delta[i] + dj) * 0.5;
    double mij = (delta[i] + dj) * (double)p->n * 0.5;
    double A = or_norm(p, kij, mij, dij);
    double Cij = 0.5 * (coef[i] + cj);
    return Cij * A * or_profile(p, sqrt((double)q) / mij);
}

static int64_t div_reach(const or_problem* p, const double* delta)
{
    int64_t N = npoints(p);
    double dmax = 0.0;
    for (int64_t i = 0; i < N; i++) if (delta[i] > dmax) dmax = delta[i];
    return isqrt_floor(or_cutoff(dmax, p->n));
}

static int64_t max_cutoff(const or_problem* p, const double* delta)
{
    int64_t N = npoints(p), km = 0;
    for (int64_t i = 0; i < N; i++) {
        int64_t k = or_cutoff(delta[i], p->n);
        if (k > km) km = k;
    }
    return km;
}

int or_apply_div(const or_problem* p, const double* delta, const double* coef,
                 const double* u, double* out)
{
    int d = p->dim;
    int64_t N = npoints(p);
    double hd = pow(1.0 / (double)p->n, (double)d);
    int64_t J = div_reach(p, delta);
    if (J > p->R) return -1;
    moment_memo mm = {0, NULL};
    if (p->norm == 0 && p->kernel <= 2) { memo_build(p, max_cutoff(p, delta), &mm); g_memo = &mm; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        int64_t x[3], y[3], z[3] = {0, 0, 0}, kij;
        unflatten(p, i, x);
        int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
        int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
        int64_t xi = pidx(p, x);
        double acc = 0.0;
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                    int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                    if (q == 0) continue;
                    for (int a = 0; a < 3; a++) y[a] = x[a] + z[a];
                    double w = div_weight(p, delta, coef, i, y, z, &kij);
                    if (q > kij) continue;
                    acc += w * (u[pidx(p, y)] - u[xi]) * hd;
                }
        out[i] = acc;
    }
    g_memo = NULL;
    free(mm.T);
    return 0;
}

/* Diagonal of -L (case b) with a zero collar: sum_j omega_ij h^d. */
int or_div_diag(const or_problem* p, const double* delta, const double* coef, double* diag)
{
    int d = p->dim;
    int64_t N = npoints(p);
    double hd = pow(1.0 / (double)p->n, (double)d);
    int64_t J = div_reach(p, delta);
    moment_memo mm = {0, NULL};
    if (p->norm == 0 && p->kernel <= 2) { memo_build(p, max_cutoff(p, delta), &mm); g_memo = &mm; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        int64_t x[3], y[3], z[3] = {0, 0, 0}, kij;
        unflatten(p, i, x);
        int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
        int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
        double acc = 0.0;
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                    int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                    if (q == 0) continue;
                    for (int a = 0; a < 3; a++) y[a] = x[a] + z[a];
                    double w = div_weight(p, delta, coef, i, y, z, &kij);
                    if (q > kij) continue;
                    acc += w * hd;
                }
        diag[i] = acc;
    }
    g_memo = NULL;
    free(mm.T);
    return 0;
}

/* ------------------------------------------------------------------ kernel-averaged form */
/* The symmetric operator with the average of the two case (a) kernels of a
 * pair (cases (a) and (b) of Section 2: the case (a) weight omega_x(y) =
 * c_x A_x g(|z|/m_x) on the ball of x; averaging it with omega_y(x) makes the
 * pair weight symmetric):
 *   L u_i = sum_{z != 0} w_s(i, i+z) (u_{i+z} - u_i) h^d,
 *   w_s(i, j) = (omega_i(j) + omega_j(i)) / 2 for j in Omega,
 *   w_s(i, j) = omega_i(j) for j in the collar.
 * diag != NULL: writes sum_j w_s(i, j) h^d (the diagonal of -L) instead. */
static double nd_weight(const or_problem* p, const double* delta, const double* coef, int64_t i, int64_t q)
{
    int64_t k = or_cutoff(delta[i], p->n);
    if (q > k) return 0.0;
    double m = delta[i] * (double)p->n;
    return coef[i] * or_norm(p, k, m, delta[i]) * or_profile(p, sqrt((double)q) / m);
}

static int sym_apply(const or_problem* p, const double* delta, const double* coef, const double* u,
                     double* out, int diag)
{
    int d = p->dim;
    int64_t N = npoints(p);
    double hd = pow(1.0 / (double)p->n, (double)d);
    int64_t J = div_reach(p, delta);
    if (J > p->R) return -1;
    moment_memo mm = {0, NULL};
    if (p->norm == 0 && p->kernel <= 2) { memo_build(p, max_cutoff(p, delta), &mm); g_memo = &mm; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        int64_t x[3], y[3], z[3] = {0, 0, 0};
        unflatten(p, i, x);
        int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
        int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
        int64_t xi = pidx(p, x);
        double acc = 0.0;
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++) {
                    int64_t q = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                    if (q == 0) continue;
                    for (int a = 0; a < 3; a++) y[a] = x[a] + z[a];
                    double w = nd_weight(p, delta, coef, i, q);
                    if (in_omega(p, y)) w = 0.5 * (w + nd_weight(p, delta, coef, gidx(p, y), q));
                    if (w == 0.0) continue;
                    acc += diag ? w * hd : w * (u[pidx(p, y)] - u[xi]) * hd;
                }
        out[i] = acc;
    }
    g_memo = NULL;
    free(mm.T);
    return 0;
}

int or_apply_sym(const or_problem* p, const double* delta, const double* coef, const double* u, double* out)
{
    return sym_apply(p, delta, coef, u, out, 0);
}

int or_sym_diag(const or_problem* p, const double* delta, const double* coef, double* diag)
{
    return sym_apply(p, delta, coef, NULL, diag, 1);
}

/* ------------------------------------------------------------------ Section 3 */
/* Step 1 (Algorithm "recur" with the cube/ball test of Algorithm
 * "doesCubeIntersectBall"), on the dyadic tree over Omega with L levels below
 * the root, 2^L >= n.  Panel (l, j) covers the node box
 * j_a 2^(L-l) .. (j_a+1) 2^(L-l) - 1 on each axis.  Geometry is taken on node
 * boxes: a panel is fully contained when it lies in Omega and all 2^d corner
 * nodes are in the lattice ball; it meets the ball when the nearest node of
 * its (Omega-clipped) box is in the ball, i.e. the clamped squared distance of
 * the intersection test is < k + 1. */
typedef struct {
    int dim;
    int64_t n;
    int L;
    int64_t c[3];
    int64_t k;
    int64_t count, cap;
    int* lev;
    int64_t* idx; /* dim entries per panel */
} dec_ctx;

/* Algorithm "doesCubeIntersectBall": squared distance from C to the box,
 * compared with r^2. */
static int cube_meets_ball(int d, const int64_t* bmin, const int64_t* bmax, const int64_t* C,
                           int64_t r2)
{
    int64_t dmin = 0;
    for (int i = 0; i < d; i++) {
        if (bmin[i] > C[i]) dmin += (bmin[i] - C[i]) * (bmin[i] - C[i]);
        else if (bmax[i] < C[i]) dmin += (bmax[i] - C[i]) * (bmax[i] - C[i]);
    }
    return dmin < r2;
}

static int in_ball(const dec_ctx* c, const int64_t* y)
{
    int64_t q = 0;
    for (int a = 0; a < c->dim; a++) q += (y[a] - c->c[a]) * (y[a] - c->c[a]);
    return q <= c->k;
}

static void include_panel(dec_ctx* c, int l, const int64_t* j)
{
    if (c->count < c->cap) {
        c->lev[c->count] = l;
        for (int a = 0; a < c->dim; a++) c->idx[c->count * c->dim + a] = j[a];
    }
    c->count++;
}

static int recur(dec_ctx* c, int l, const int64_t* j)
{
    int d = c->dim;
    int64_t side = (int64_t)1 << (c->L - l);
    int64_t lo[3], hi[3];
    int inside_omega = 1;
    for (int a = 0; a < d; a++) {
        lo[a] = j[a] * side;
        hi[a] = lo[a] + side - 1;
        if (hi[a] > c->n - 1) inside_omega = 0;
    }
    /* fully contained in H_x and Omega: all 2^d corners in the ball */
    if (inside_omega) {
        int all = 1;
        for (int m = 0; m < (1 << d) && all; m++) {
            int64_t y[3];
            for (int a = 0; a < d; a++) y[a] = (m >> a & 1) ? hi[a] : lo[a];
            all = in_ball(c, y);
        }
        if (all) { include_panel(c, l, j); return 1; }
    }
    /* nontrivial intersection with H_x cut by Omega */
    int64_t chi[3];
    for (int a = 0; a < d; a++) {
        if (lo[a] > c->n - 1) return 0;
        chi[a] = hi[a] < c->n - 1 ? hi[a] : c->n - 1;
    }
    if (cube_meets_ball(d, lo, chi, c->c, c->k + 1)) {
        if (l < c->L) {
            for (int m = 0; m < (1 << d); m++) {
                int64_t jc[3];
                for (int a = 0; a < d; a++) jc[a] = 2 * j[a] + (m >> a & 1);
                recur(c, l + 1, jc);
            }
            return 0;
        }
        include_panel(c, l, j);
        return 1;
    }
    return 0;
}

int or_tree_levels(int64_t n)
{
    int L = 0;
    while (((int64_t)1 << L) < n) L++;
    return L;
}

/* Decomposition of (lattice ball of squared radius k around node `center`) cut
 * by Omega into maximal tree panels.  Writes up to `cap` panels (level and
 * dim indices each) and returns the total count. */
int64_t or_decompose(int dim, int64_t n, const int64_t* center, int64_t k,
                     int* lev, int64_t* idx, int64_t cap)
{
    dec_ctx c;
    memset(&c, 0, sizeof(c));
    c.dim = dim; c.n = n; c.L = or_tree_levels(n); c.k = k;
    for (int a = 0; a < dim; a++) c.c[a] = center[a];
    c.cap = cap; c.lev = lev; c.idx = idx;
    int64_t root[3] = {0, 0, 0};
    recur(&c, 0, root);
    return c.count;
}

/* Step 2: partial sums of u over every panel of every level, bottom-up.
 * Level l is stored as a (2^l)^dim array at offset sum_{l'<l} (2^l')^dim.
 * u is the unpadded n^dim grid; nodes of the padded tree beyond n hold 0
 * (u = 0 outside Omega). */
int64_t or_tree_size(int dim, int64_t n)
{
    int L = or_tree_levels(n);
    int64_t tot = 0;
    for (int l = 0; l <= L; l++) tot += (int64_t)1 << (dim * l);
    return tot;
}

static int64_t level_offset(int dim, int l)
{
    int64_t off = 0;
    for (int q = 0; q < l; q++) off += (int64_t)1 << (dim * q);
    return off;
}

void or_partial_sums(int dim, int64_t n, const double* u, double* S)
{
    int L = or_tree_levels(n);
    int64_t side = (int64_t)1 << L;
    double* leaf = S + level_offset(dim, L);
    int64_t cnt = (int64_t)1 << (dim * L);
    for (int64_t t = 0; t < cnt; t++) {
        int64_t x[3] = {0, 0, 0}, r = t, ok = 1, g = 0;
        for (int a = dim - 1; a >= 0; a--) { x[a] = r % side; r /= side; }
        for (int a = 0; a < dim; a++) { if (x[a] >= n) ok = 0; g = g * n + x[a]; }
        leaf[t] = ok ? u[g] : 0.0;
    }
    for (int l = L - 1; l >= 0; l--) {
        double* par = S + level_offset(dim, l);
        double* chi = S + level_offset(dim, l + 1);
        int64_t ps = (int64_t)1 << l, cs = ps * 2;
        int64_t pc = (int64_t)1 << (dim * l);
        for (int64_t t = 0; t < pc; t++) {
            int64_t j[3] = {0, 0, 0}, r = t;
            for (int a = dim - 1; a >= 0; a--) { j[a] = r % ps; r /= ps; }
            double acc = 0.0;
            for (int m = 0; m < (1 << dim); m++) {
                int64_t ci = 0;
                for (int a = 0; a < dim; a++) ci = ci * cs + (2 * j[a] + (m >> a & 1));
                acc += chi[ci];
            }
            par[t] = acc;
        }
    }
}

/* The three steps of Section 3 for the truncated constant profile (K = 0,
 * p^0 = 1), zero volume constraint, case (a) with C = c(x), delta = delta(x):
 *   L^P u_i = c_i A_i h^d ( sum_{panels of H_i cut by Omega} S_panel - M_i u_i ),
 * eq. "nonlocalP" with |H_x| = M_i h^d, M_i = #{z : |z|^2 <= k_i}.  The
 * problem must have kernel 0.  u is the unpadded grid. */
int or_fast_apply_const(const or_problem* p, const double* delta, const double* coef,
                        const double* u, double* out)
{
    if (p->kernel != 0 || p->model != 0 || p->form != 0) return -1;
    int d = p->dim;
    int64_t n = p->n, N = npoints(p);
    double hd = pow(1.0 / (double)n, (double)d);
    int L = or_tree_levels(n);
    double* S = (double*)malloc(sizeof(double) * or_tree_size(d, n));
    if (!S) return -2;
    or_partial_sums(d, n, u, S); /* Step 2 */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; i++) {
        int64_t x[3];
        unflatten(p, i, x);
        int64_t k = or_cutoff(delta[i], n);
        /* Step 1 for this node (the paper stores it; recomputing is the same list) */
        int64_t cap = 4096, cnt;
        int* lev = NULL; int64_t* idx = NULL;
        for (;;) {
            lev = (int*)malloc(sizeof(int) * cap);
            idx = (int64_t*)malloc(sizeof(int64_t) * cap * d);
            cnt = or_decompose(d, n, x, k, lev, idx, cap);
            if (cnt <= cap) break;
            free(lev); free(idx); cap = cnt;
        }
        /* Step 3: sum of the stored partial sums over the decomposition */
        double sum = 0.0;
        for (int64_t q = 0; q < cnt; q++) {
            int l = lev[q];
            int64_t side = (int64_t)1 << l, off = 0;
            for (int a = 0; a < d; a++) off = off * side + idx[q * d + a];
            sum += S[level_offset(d, l) + off];
        }
        free(lev); free(idx);
        int64_t J = isqrt_floor(k), M = 0;
        int64_t z[3] = {0, 0, 0};
        int64_t lo1 = d >= 2 ? -J : 0, hi1 = d >= 2 ? J : 0;
        int64_t lo2 = d >= 3 ? -J : 0, hi2 = d >= 3 ? J : 0;
        for (z[0] = -J; z[0] <= J; z[0]++)
            for (z[1] = lo1; z[1] <= hi1; z[1]++)
                for (z[2] = lo2; z[2] <= hi2; z[2]++)
                    if (z[0] * z[0] + z[1] * z[1] + z[2] * z[2] <= k) M++;
        double m = delta[i] * (double)n;
        double A = or_norm(p, k, m, delta[i]);
        out[i] = coef[i] * A * hd * (sum - (double)M * u[i]);
    }
    (void)L;
    free(S);
    return 0;
}

/* ------------------------------------------------------------------ solve */
/* Conjugate gradients (optionally Jacobi-preconditioned) for -L x = b in case
 * (b) with zero volume constraint; the stopping rule is the true FP64 relative
 * residual ||b + L x|| / ||b|| <= rtol.  x holds the start value on entry. */
static void div_matvec(const or_problem* p, const double* delta, const double* coef,
                       const double* x, double* ax, double* pad)
{
    int64_t N = npoints(p);
    int64_t Pn = 1;
    for (int a = 0; a < p->dim; a++) Pn *= (p->n + 2 * p->R);
    memset(pad, 0, sizeof(double) * Pn);
    for (int64_t i = 0; i < N; i++) {
        int64_t xx[3];
        unflatten(p, i, xx);
        pad[pidx(p, xx)] = x[i];
    }
    or_apply_div(p, delta, coef, pad, ax);
    for (int64_t i = 0; i < N; i++) ax[i] = -ax[i];
}

static double dot(const double* a, const double* b, int64_t N)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; i++) s += a[i] * b[i];
    return s;
}

int or_cg_div(const or_problem* p, const double* delta, const double* coef, const double* b,
              double* x, double rtol, int maxit, int jacobi, int* iters, double* relres)
{
    int64_t N = npoints(p);
    int64_t Pn = 1;
    for (int a = 0; a < p->dim; a++) Pn *= (p->n + 2 * p->R);
    if (div_reach(p, delta) > p->R) return -1;
    double* r = (double*)malloc(sizeof(double) * N);
    double* z = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    double* d = (double*)malloc(sizeof(double) * N);
    double* dg = (double*)malloc(sizeof(double) * N);
    double* pad = (double*)malloc(sizeof(double) * Pn);
    or_div_diag(p, delta, coef, dg);
    double bn = sqrt(dot(b, b, N));
    div_matvec(p, delta, coef, x, q, pad);
    for (int64_t i = 0; i < N; i++) r[i] = b[i] - q[i];
    for (int64_t i = 0; i < N; i++) z[i] = jacobi ? r[i] / dg[i] : r[i];
    memcpy(d, z, sizeof(double) * N);
    double rz = dot(r, z, N);
    int it = 0, ok = 0;
    double rel = sqrt(dot(r, r, N)) / bn;
    if (rel <= rtol) ok = 1;
    while (!ok && it < maxit) {
        div_matvec(p, delta, coef, d, q, pad);
        double alpha = rz / dot(d, q, N);
        for (int64_t i = 0; i < N; i++) { x[i] += alpha * d[i]; r[i] -= alpha * q[i]; }
        it++;
        if (sqrt(dot(r, r, N)) / bn <= rtol) {
            div_matvec(p, delta, coef, x, q, pad); /* confirm with the true residual */
            double tr = 0.0;
            for (int64_t i = 0; i < N; i++) tr += (b[i] - q[i]) * (b[i] - q[i]);
            rel = sqrt(tr) / bn;
            if (rel <= rtol) { ok = 1; break; }
        }
        for (int64_t i = 0; i < N; i++) z[i] = jacobi ? r[i] / dg[i] : r[i];
        double rz2 = dot(r, z, N);
        double beta = rz2 / rz;
        rz = rz2;
        for (int64_t i = 0; i < N; i++) d[i] = z[i] + beta * d[i];
    }
    if (!ok) {
        div_matvec(p, delta, coef, x, q, pad);
        double tr = 0.0;
        for (int64_t i = 0; i < N; i++) tr += (b[i] - q[i]) * (b[i] - q[i]);
        rel = sqrt(tr) / bn;
    }
    *iters = it;
    *relres = rel;
    free(r); free(z); free(q); free(d); free(dg); free(pad);
    return ok ? 0 : 1;
}
