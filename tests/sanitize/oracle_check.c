/*
 * sanitize_main.c -- TEST INFRASTRUCTURE.  A driver that runs every function of the oracle
 * (lm_oracle.c) on small inputs so that the oracle can be built and run under the host
 * sanitizers (AddressSanitizer and UndefinedBehaviorSanitizer): out-of-bounds indexing,
 * use after free, leaks, signed overflow and invalid shifts in the oracle show up as a
 * sanitizer report and a non-zero exit status.  Built and run by the CPU test suite.
 *
 * The cases cover the sizes where index arithmetic is most likely to slip: one particle,
 * two coincident particles, ragged sizes, 2-D and 3-D, both kernels, tau > 0, sampled rows
 * with repeated and unsorted indices, and a number of passive points different from the
 * number of particles.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void orc_rhs(int dim, long n, int kernel, double sigma, double tau, const double *q, const double *p, double *dq,
             double *dp);
void orc_rhs_rows(int dim, long n, int kernel, double sigma, double tau, const double *q, const double *p,
                  const long *idx, long nidx, double *dq_rows, double *dp_rows);
double orc_hamiltonian(int dim, long n, int kernel, double sigma, const double *q, const double *p);
void orc_shoot(int dim, long n, int kernel, double sigma, double tau, double T, int steps, const double *q0,
               const double *p0, double *q1, double *p1);
void orc_kmatrix(int dim, long n, int kernel, double sigma, const double *X, double *K);
int orc_cholesky(long n, double *A);
void orc_cholesky_solve(long n, const double *L, const double *b, double *x);
int orc_feedback_match(int dim, long n, int kernel, double sigma, double tau, const double *X, const double *Y,
                       double h, double tol, int max_iter, int steps, int stop_rule, double *p0, double *q1_out,
                       int *iters, double *resid, double *H, double *hist, int hist_len);
void orc_rhs_vjp(int dim, long n, int kernel, double sigma, double tau, const double *q, const double *p,
                 const double *a, const double *b, double *aq, double *ap);
void orc_shoot_adjoint(int dim, long n, int kernel, double sigma, double tau, double T, int steps,
                       const double *q0, const double *p0, const double *gq1, const double *gp1, double *gq0,
                       double *gp0);
void orc_velocity(int dim, long n, long m, int kernel, double sigma, const double *q, const double *p,
                  const double *x, double *u);
void orc_flow_points(int dim, long n, long m, int kernel, double sigma, double tau, double T, int steps,
                     const double *q0, const double *p0, const double *x0, double *q1, double *p1, double *x1);

static unsigned long long g_state = 88172645463325252ULL;

/* xorshift64: deterministic filler values in [-1, 1) */
static double rnd(void)
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double *arr(size_t count, double scale)
{
    double *a = (double *)malloc(sizeof(double) * (count ? count : 1));
    for (size_t k = 0; k < count; ++k) a[k] = scale * rnd();
    return a;
}

static int g_bad = 0;

static void check_finite(const char *what, const double *a, size_t count)
{
    for (size_t k = 0; k < count; ++k)
        if (!isfinite(a[k])) {
            fprintf(stderr, "%s: non-finite value at %zu\n", what, k);
            g_bad = 1;
            return;
        }
}

static void run_case(int dim, long n, long m, int kernel, double tau)
{
    const double sigma = 0.4;
    size_t sz = (size_t)dim * (size_t)n, sx = (size_t)dim * (size_t)m;
    double *q = arr(sz, 1.0), *p = arr(sz, 0.3), *a = arr(sz, 1.0), *b = arr(sz, 1.0), *x = arr(sx, 1.2);
    if (n >= 2)
        for (int c = 0; c < dim; ++c) q[c * n + 1] = q[c * n + 0];      /* two coincident particles */
    double *dq = arr(sz, 0.0), *dp = arr(sz, 0.0), *q1 = arr(sz, 0.0), *p1 = arr(sz, 0.0), *x1 = arr(sx, 0.0);
    double *aq = arr(sz, 0.0), *ap = arr(sz, 0.0);

    orc_rhs(dim, n, kernel, sigma, tau, q, p, dq, dp);
    check_finite("rhs", dp, sz);

    long nidx = 5;
    long idx[5] = {n - 1, 0, n / 2, 0, n - 1};                         /* unsorted, repeated */
    double *rq = arr((size_t)dim * nidx, 0.0), *rp = arr((size_t)dim * nidx, 0.0);
    orc_rhs_rows(dim, n, kernel, sigma, tau, q, p, idx, nidx, rq, rp);
    for (long k = 0; k < nidx; ++k)
        for (int c = 0; c < dim; ++c)
            if (rq[c * nidx + k] != dq[c * n + idx[k]] || rp[c * nidx + k] != dp[c * n + idx[k]]) {
                fprintf(stderr, "rhs_rows differs from rhs at row %ld\n", idx[k]);
                g_bad = 1;
            }

    double H = orc_hamiltonian(dim, n, kernel, sigma, q, p);
    check_finite("hamiltonian", &H, 1);

    orc_shoot(dim, n, kernel, sigma, tau, 0.7, 3, q, p, q1, p1);
    check_finite("shoot", q1, sz);

    orc_velocity(dim, n, m, kernel, sigma, q, p, x, x1);
    check_finite("velocity", x1, sx);

    orc_flow_points(dim, n, m, kernel, sigma, tau, 0.7, 3, q, p, x, q1, p1, x1);
    check_finite("flow_points", x1, sx);

    orc_rhs_vjp(dim, n, kernel, sigma, tau, q, p, a, b, aq, ap);
    check_finite("rhs_vjp", aq, sz);
    orc_shoot_adjoint(dim, n, kernel, sigma, tau, 0.7, 3, q, p, a, b, aq, ap);
    check_finite("shoot_adjoint", ap, sz);

    /* Algorithm 1 and the K-solve on distinct points (a coincident pair makes K singular) */
    for (int c = 0; c < dim; ++c)
        for (long i = 0; i < n; ++i) q[c * n + i] = (c == 0 ? 0.5 : 0.25) * (double)i + 0.1 * rnd();
    double *K = arr((size_t)n * (size_t)n, 0.0), *y = arr((size_t)n, 0.0);
    orc_kmatrix(dim, n, kernel, sigma, q, K);
    if (orc_cholesky(n, K) == 0) {
        orc_cholesky_solve(n, K, a, y);
        check_finite("cholesky_solve", y, (size_t)n);
    }
    double *Y = arr(sz, 0.0), *p0 = arr(sz, 0.0), hist[16];
    for (size_t k = 0; k < sz; ++k) {
        Y[k] = q[k] + 0.01 * rnd();
        p0[k] = 0.0;
    }
    int iters = 0;
    double resid = 0.0, Hm = 0.0;
    orc_feedback_match(dim, n, kernel, sigma, tau, q, Y, 0.8, 1e-6, 40, 4, tau > 0.0 ? 1 : 0, p0, q1, &iters, &resid,
                       &Hm, hist, 16);
    check_finite("feedback_match", p0, sz);

    free(q); free(p); free(a); free(b); free(x); free(dq); free(dp); free(q1); free(p1); free(x1);
    free(aq); free(ap); free(rq); free(rp); free(K); free(y); free(Y); free(p0);
}

int main(void)
{
    const long sizes[] = {1, 2, 3, 17, 65};
    for (int dim = 2; dim <= 3; ++dim)
        for (int kernel = 0; kernel <= 1; ++kernel)
            for (int s = 0; s < 5; ++s) {
                run_case(dim, sizes[s], sizes[(s + 2) % 5], kernel, 0.0);
                run_case(dim, sizes[s], sizes[(s + 1) % 5], kernel, 0.2);
            }
    if (g_bad) return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
