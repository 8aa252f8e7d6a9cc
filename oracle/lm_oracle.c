/*
 * lm_oracle.c -- plain FP64 CPU oracle of geodesic landmark shooting with the N-particle
 * Euler-Poincare system (Camassa, Kuang & Lee, arXiv 1510.03816).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU library is compared against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the GPU library neither links nor calls it
 * and the two share no code.
 *
 * Conventions
 *   - every array is float64, component-major: x[c*n + i] is coordinate c of landmark i;
 *   - kernel 0 = conical ("conon") G(r) = exp(-r/sigma): the normalised Green's function
 *     of the operator (I - sigma^2 Laplacian)^(3/2) in the plane (equation of the conon and
 *     the normalisation stated at the start of the exact-matching experiments);
 *     kernel 1 = Gaussian G(r) = exp(-r^2/sigma^2) (the smooth kernel "G_infinity" of the
 *     metric comparison section; its width enters as sigma^2 = alpha^2);
 *   - no FMA contraction (built with -ffp-contract=off), round-to-nearest, libm exp/sqrt;
 *   - OpenMP parallelises over the target index i only; every j-sum runs j = 0..n-1 in
 *     order, so results do not depend on the thread count.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - the self term j = i is included in the velocity sum (G(0) = 1) and excluded from the
 *     force sum, as in the N-particle system as printed;
 *   - two distinct particles at the same point exert no force on each other (the direction
 *     (q_i - q_j)/|q_i - q_j| is undefined there; zero is the mean of its one-sided limits);
 *   - Algorithm 1's "update the momenta from the velocity" is p = K(X)^{-1} u with
 *     K_ij = G(|X_i - X_j|) at the template, so with M = hI the update is
 *     p <- p + h K(X)^{-1} (Y - q(1));
 *   - the stopping norm is the maximum over all N*dim coordinates, with a strict "<";
 *   - the iteration count is the number of momentum updates made before the shoot that
 *     passes the test.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTPD (-2)
#define ORC_ENOTCONV (-4)
#define ORC_EDIVERGED (-5)

/* Threads the OpenMP loops use (reported with timings of the oracle). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- Green's functions: G(r) and its radial derivative G'(r) -------------------------- */

/* Conon (equation of G_{1/2}, normalised): G(r) = exp(-r/sigma), G'(r) = -G(r)/sigma.
 * Gaussian: G(r) = exp(-r^2/sigma^2), G'(r) = -2 r G(r)/sigma^2. */
static double green(int kernel, double sigma, double r)
{
    if (kernel == 0) return exp(-r / sigma);
    return exp(-(r * r) / (sigma * sigma));
}

static double green_prime(int kernel, double sigma, double r)
{
    if (kernel == 0) return -exp(-r / sigma) / sigma;
    return -2.0 * r * exp(-(r * r) / (sigma * sigma)) / (sigma * sigma);
}

/* G'(r) given g = G(r), to evaluate the exponential once per pair. */
static double green_prime_g(int kernel, double sigma, double r, double g)
{
    if (kernel == 0) return -g / sigma;
    return -2.0 * r * g / (sigma * sigma);
}

double orc_green(int kernel, double sigma, double r) { return green(kernel, sigma, r); }
double orc_green_prime(int kernel, double sigma, double r) { return green_prime(kernel, sigma, r); }

static double dist(int dim, long n, const double *q, long i, long j)
{
    double s = 0.0;
    for (int c = 0; c < dim; ++c) {
        double d = q[c * n + i] - q[c * n + j];
        s += d * d;
    }
    return sqrt(s);
}

/* ---- The N-particle system (equation "N-particle"; tau > 0 adds the tau*p_i advection of
 * the inexact system, equation "N-particle-inexact", where the paper calls tau sigma^2) ---
 *
 *   dq_i/dt =  sum_{j=1..N} G(|q_i - q_j|) p_j + tau p_i
 *   dp_i/dt = -sum_{j != i} (p_i . p_j) G'(|q_i - q_j|) (q_i - q_j)/|q_i - q_j|
 */
void orc_rhs(int dim, long n, int kernel, double sigma, double tau,
             const double *q, const double *p, double *dq, double *dp)
{
#pragma omp parallel for schedule(static) if (n >= 256)
    for (long i = 0; i < n; ++i) {
        double v[3] = {0.0, 0.0, 0.0}, f[3] = {0.0, 0.0, 0.0};
        for (long j = 0; j < n; ++j) {
            double r = dist(dim, n, q, i, j);
            double g = green(kernel, sigma, r);
            for (int c = 0; c < dim; ++c) v[c] += g * p[c * n + j];
            if (j == i || r == 0.0) continue;
            double pp = 0.0;
            for (int c = 0; c < dim; ++c) pp += p[c * n + i] * p[c * n + j];
            double gp = green_prime_g(kernel, sigma, r, g);
            for (int c = 0; c < dim; ++c)
                f[c] -= pp * gp * (q[c * n + i] - q[c * n + j]) / r;
        }
        for (int c = 0; c < dim; ++c) {
            dq[c * n + i] = v[c] + tau * p[c * n + i];
            dp[c * n + i] = f[c];
        }
    }
}

/* The same right-hand side for a subset of targets: rows idx[0..nidx) of (dq, dp), written
 * to dq_rows/dp_rows as (dim, nidx).  Lets large problems be checked on sampled outputs. */
void orc_rhs_rows(int dim, long n, int kernel, double sigma, double tau,
                  const double *q, const double *p, const long *idx, long nidx,
                  double *dq_rows, double *dp_rows)
{
#pragma omp parallel for schedule(static) if (nidx >= 16)
    for (long a = 0; a < nidx; ++a) {
        long i = idx[a];
        double v[3] = {0.0, 0.0, 0.0}, f[3] = {0.0, 0.0, 0.0};
        for (long j = 0; j < n; ++j) {
            double r = dist(dim, n, q, i, j);
            double g = green(kernel, sigma, r);
            for (int c = 0; c < dim; ++c) v[c] += g * p[c * n + j];
            if (j == i || r == 0.0) continue;
            double pp = 0.0;
            for (int c = 0; c < dim; ++c) pp += p[c * n + i] * p[c * n + j];
            double gp = green_prime_g(kernel, sigma, r, g);
            for (int c = 0; c < dim; ++c)
                f[c] -= pp * gp * (q[c * n + i] - q[c * n + j]) / r;
        }
        for (int c = 0; c < dim; ++c) {
            dq_rows[c * nidx + a] = v[c] + tau * p[c * n + i];
            dp_rows[c * nidx + a] = f[c];
        }
    }
}

/* ---- Discrete Hamiltonian (equation "H"): H = 1/2 sum_i sum_j (p_i . p_j) G(|q_i - q_j|).
 * The Hamiltonian values printed with the examples are 2H (the energy E of eq. "E=2H"). */
double orc_hamiltonian(int dim, long n, int kernel, double sigma, const double *q, const double *p)
{
    double *row = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static) if (n >= 256)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (long j = 0; j < n; ++j) {
            double pp = 0.0;
            for (int c = 0; c < dim; ++c) pp += p[c * n + i] * p[c * n + j];
            s += pp * green(kernel, sigma, dist(dim, n, q, i, j));
        }
        row[i] = s;
    }
    double H = 0.0;
    for (long i = 0; i < n; ++i) H += row[i];
    free(row);
    return 0.5 * H;
}

/* ---- Shooting map: the classical fourth-order Runge-Kutta method on t in [0, T] with
 * `steps` equal steps (an explicit integrator of the kind the paper names; the flow is
 * evolved to t = 1 in Algorithm 1). ------------------------------------------------------ */
void orc_shoot(int dim, long n, int kernel, double sigma, double tau, double T, int steps,
               const double *q0, const double *p0, double *q1, double *p1)
{
    size_t m = (size_t)dim * (size_t)n;
    double *q = (double *)malloc(sizeof(double) * m), *p = (double *)malloc(sizeof(double) * m);
    double *qs = (double *)malloc(sizeof(double) * m), *ps = (double *)malloc(sizeof(double) * m);
    double *kq[4], *kp[4];
    for (int s = 0; s < 4; ++s) {
        kq[s] = (double *)malloc(sizeof(double) * m);
        kp[s] = (double *)malloc(sizeof(double) * m);
    }
    memcpy(q, q0, sizeof(double) * m);
    memcpy(p, p0, sizeof(double) * m);
    double dt = T / steps;
    const double cstage[4] = {0.0, 0.5, 0.5, 1.0};
    for (int step = 0; step < steps; ++step) {
        for (int s = 0; s < 4; ++s) {
            if (s == 0) {
                orc_rhs(dim, n, kernel, sigma, tau, q, p, kq[0], kp[0]);
            } else {
                for (size_t k = 0; k < m; ++k) {
                    qs[k] = q[k] + cstage[s] * dt * kq[s - 1][k];
                    ps[k] = p[k] + cstage[s] * dt * kp[s - 1][k];
                }
                orc_rhs(dim, n, kernel, sigma, tau, qs, ps, kq[s], kp[s]);
            }
        }
        for (size_t k = 0; k < m; ++k) {
            q[k] = q[k] + dt / 6.0 * (kq[0][k] + 2.0 * kq[1][k] + 2.0 * kq[2][k] + kq[3][k]);
            p[k] = p[k] + dt / 6.0 * (kp[0][k] + 2.0 * kp[1][k] + 2.0 * kp[2][k] + kp[3][k]);
        }
    }
    memcpy(q1, q, sizeof(double) * m);
    memcpy(p1, p, sizeof(double) * m);
    free(q); free(p); free(qs); free(ps);
    for (int s = 0; s < 4; ++s) { free(kq[s]); free(kp[s]); }
}

/* ---- Kernel matrix K_ij = G(|X_i - X_j|), row-major n x n. ------------------------------ */
void orc_kmatrix(int dim, long n, int kernel, double sigma, const double *X, double *K)
{
#pragma omp parallel for schedule(static) if (n >= 256)
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j)
            K[i * n + j] = green(kernel, sigma, dist(dim, n, X, i, j));
}

/* Textbook Cholesky A = L L^T, L overwrites the lower triangle of A (row-major).
 * Returns ORC_ENOTPD when a pivot is not positive. */
int orc_cholesky(long n, double *A)
{
    for (long j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (long k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0)) return ORC_ENOTPD;
        double ljj = sqrt(d);
        A[j * n + j] = ljj;
#pragma omp parallel for schedule(static) if (n - j >= 512)
        for (long i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (long k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / ljj;
        }
    }
    return ORC_OK;
}

/* Solve L L^T x = b with the factor from orc_cholesky (forward then back substitution). */
void orc_cholesky_solve(long n, const double *L, const double *b, double *x)
{
    for (long i = 0; i < n; ++i) {
        double s = b[i];
        for (long k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
        x[i] = s / L[i * n + i];
    }
    for (long i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (long k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

static double max_abs_diff(size_t m, const double *a, const double *b)
{
    double r = 0.0;
    for (size_t k = 0; k < m; ++k) {
        double e = fabs(a[k] - b[k]);
        if (e != e) return e;          /* propagate NaN */
        if (e > r) r = e;
    }
    return r;
}

/* ---- Algorithm 1 (feedback-control iteration) with M = h I -------------------------------
 *
 *   factor K(X) (with tau on its diagonal for the inexact system: the t = 0 velocity of the
 *   inexact system is (K + tau I) p);  p <- p0 (zeros in the paper);
 *   for k = 0, 1, ...:
 *       q1 = shoot(X, p) to t = 1;  e = Y - q1
 *       exact  (stop_rule 0): stop when max|e| < tol
 *       inexact(stop_rule 1): stop when max|u^k - u^{k-1}| < tol, i.e. h*max|e^{k-1}| < tol
 *                             (the rule stated with the inexact-matching table), k >= 1
 *       u <- u + h e, i.e. p <- p + h (K + tau I)^{-1} e
 *
 * Returns ORC_OK, ORC_ENOTCONV (max_iter updates made without meeting tol), ORC_EDIVERGED
 * (non-finite residual) or ORC_ENOTPD (K not numerically positive definite).  On return p0
 * holds the last momenta, *iters the number of updates made, *resid the max-norm residual
 * of the last shoot, *H the Hamiltonian (1/2 form) at (X, p0).  hist (nullable) receives the
 * residual of every shoot, up to hist_len entries. */
int orc_feedback_match(int dim, long n, int kernel, double sigma, double tau,
                       const double *X, const double *Y, double h, double tol,
                       int max_iter, int steps, int stop_rule,
                       double *p0, double *q1_out, int *iters, double *resid, double *H,
                       double *hist, int hist_len)
{
    if (dim < 1 || n < 1 || !(sigma > 0.0) || !(h > 0.0) || !(tol > 0.0) || steps < 1 || max_iter < 0)
        return ORC_EINVAL;
    size_t m = (size_t)dim * (size_t)n;
    double *K = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *q1 = (double *)malloc(sizeof(double) * m), *p1 = (double *)malloc(sizeof(double) * m);
    double *e = (double *)malloc(sizeof(double) * m), *dp = (double *)malloc(sizeof(double) * (size_t)n);
    orc_kmatrix(dim, n, kernel, sigma, X, K);
    for (long i = 0; i < n; ++i) K[i * n + i] += tau;
    int st = orc_cholesky(n, K);
    double r = 0.0, prev_step = INFINITY;
    int k = 0;
    if (st == ORC_OK) {
        for (k = 0;; ++k) {
            orc_shoot(dim, n, kernel, sigma, tau, 1.0, steps, X, p0, q1, p1);
            r = max_abs_diff(m, Y, q1);
            if (hist && k < hist_len) hist[k] = r;
            if (!isfinite(r)) { st = ORC_EDIVERGED; break; }
            if (stop_rule == 0 ? (r < tol) : (k >= 1 && prev_step < tol)) { st = ORC_OK; break; }
            if (k >= max_iter) { st = ORC_ENOTCONV; break; }
            for (size_t t = 0; t < m; ++t) e[t] = Y[t] - q1[t];
            for (int c = 0; c < dim; ++c) {
                orc_cholesky_solve(n, K, e + (size_t)c * n, dp);
                for (long i = 0; i < n; ++i) p0[c * n + i] += h * dp[i];
            }
            prev_step = h * r;
        }
    }
    if (iters) *iters = k;
    if (resid) *resid = r;
    if (q1_out) memcpy(q1_out, q1, sizeof(double) * m);
    if (H) *H = orc_hamiltonian(dim, n, kernel, sigma, X, p0);
    free(K); free(q1); free(p1); free(e); free(dp);
    return st;
}

/* ---- Reverse mode (the adjoint of the shooting map; not in the paper: it differentiates the
 * inexact-matching energy of equation "inexact-E" with respect to the initial momenta). ---
 *
 * Vector-Jacobian product of the right-hand side at (q, p): given the cotangent (a, b) of
 * (dq/dt, dp/dt), returns (aq, ap) = J^T (a, b).  With w = -G'(r)/r, u = w'(r)/r,
 * d = q_k - q_j and e = b_k - b_j, differentiating the N-particle sums gives
 *   ap_k = tau a_k + sum_j G_kj a_j + sum_{j != k} w (e . d) p_j
 *   aq_k = sum_{j != k} [ -w ((a_k . p_j) + (a_j . p_k)) d + (p_k . p_j) (w e + (e . d) u d) ]
 * (coincident distinct particles contribute nothing, as in the forward sums). */
static double wfun(int kernel, double sigma, double r, double g)
{
    return -green_prime_g(kernel, sigma, r, g) / r;
}

/* u = w'(r)/r: conon w = G/(sigma r), w' = -G/(sigma^2 r) - G/(sigma r^2);
 * Gaussian w = 2G/sigma^2, w' = -4 r G/sigma^4. */
static double ufun(int kernel, double sigma, double r, double g)
{
    if (kernel == 0) return (-g / (sigma * sigma * r) - g / (sigma * r * r)) / r;
    return -4.0 * g / (sigma * sigma * sigma * sigma);
}

void orc_rhs_vjp(int dim, long n, int kernel, double sigma, double tau,
                 const double *q, const double *p, const double *a, const double *b,
                 double *aq, double *ap)
{
#pragma omp parallel for schedule(static) if (n >= 256)
    for (long k = 0; k < n; ++k) {
        double gq[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0};
        for (long j = 0; j < n; ++j) {
            double r = dist(dim, n, q, k, j);
            double g = green(kernel, sigma, r);
            for (int c = 0; c < dim; ++c) gp[c] += g * a[c * n + j];
            if (j == k || r == 0.0) continue;
            double w = wfun(kernel, sigma, r, g), u = ufun(kernel, sigma, r, g);
            double d[3], e[3], ed = 0.0, apj = 0.0, pp = 0.0;
            for (int c = 0; c < dim; ++c) {
                d[c] = q[c * n + k] - q[c * n + j];
                e[c] = b[c * n + k] - b[c * n + j];
                ed += e[c] * d[c];
                apj += a[c * n + k] * p[c * n + j] + a[c * n + j] * p[c * n + k];
                pp += p[c * n + k] * p[c * n + j];
            }
            for (int c = 0; c < dim; ++c) {
                gp[c] += w * ed * p[c * n + j];
                gq[c] += -w * apj * d[c] + pp * (w * e[c] + ed * u * d[c]);
            }
        }
        for (int c = 0; c < dim; ++c) {
            aq[c * n + k] = gq[c];
            ap[c * n + k] = gp[c] + tau * a[c * n + k];
        }
    }
}

/* Discrete adjoint of orc_shoot: (gq0, gp0) = J_shoot^T (gq1, gp1), every stage input kept.
 * For one RK4 step y' = y + dt/6 (k1 + 2k2 + 2k3 + k4), k_s = f(Y_s), with cotangent abar of
 * y': kb4 = dt/6 abar, Yb4 = J(Y4)^T kb4; kb3 = dt/3 abar + dt Yb4, Yb3 = J(Y3)^T kb3;
 * kb2 = dt/3 abar + dt/2 Yb3, Yb2 = J(Y2)^T kb2; kb1 = dt/6 abar + dt/2 Yb2,
 * Yb1 = J(Y1)^T kb1; the cotangent of y is abar + Yb1 + Yb2 + Yb3 + Yb4. */
void orc_shoot_adjoint(int dim, long n, int kernel, double sigma, double tau, double T, int steps,
                       const double *q0, const double *p0, const double *gq1, const double *gp1,
                       double *gq0, double *gp0)
{
    size_t m = (size_t)dim * (size_t)n;
    size_t per = 2 * m;                       /* one state (q, p) */
    double *Ys = (double *)malloc(sizeof(double) * per * 4 * (size_t)steps);
    double *y = (double *)malloc(sizeof(double) * per), *ks = (double *)malloc(sizeof(double) * per * 4);
    double dt = T / steps;
    const double cst[4] = {0.0, 0.5, 0.5, 1.0};
    memcpy(y, q0, sizeof(double) * m);
    memcpy(y + m, p0, sizeof(double) * m);
    for (int st = 0; st < steps; ++st) {
        for (int s = 0; s < 4; ++s) {
            double *Y = Ys + ((size_t)st * 4 + s) * per;
            for (size_t k = 0; k < per; ++k) Y[k] = y[k] + (s ? cst[s] * dt * ks[(s - 1) * per + k] : 0.0);
            orc_rhs(dim, n, kernel, sigma, tau, Y, Y + m, ks + s * per, ks + s * per + m);
        }
        for (size_t k = 0; k < per; ++k)
            y[k] = y[k] + dt / 6.0 * (ks[k] + 2.0 * ks[per + k] + 2.0 * ks[2 * per + k] + ks[3 * per + k]);
    }
    double *lam = (double *)malloc(sizeof(double) * per), *acc = (double *)malloc(sizeof(double) * per);
    double *kb = (double *)malloc(sizeof(double) * per), *Yb = (double *)malloc(sizeof(double) * per);
    memcpy(lam, gq1, sizeof(double) * m);
    memcpy(lam + m, gp1, sizeof(double) * m);
    const double ca[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};   /* weights of abar in kb1..kb4 */
    const double cy[4] = {0.5, 0.5, 1.0, 0.0};                           /* weight of Yb_{s+1} in kb_s */
    for (int st = steps - 1; st >= 0; --st) {
        memcpy(acc, lam, sizeof(double) * per);
        for (int s = 3; s >= 0; --s) {
            for (size_t k = 0; k < per; ++k) kb[k] = dt * ca[s] * lam[k] + (s < 3 ? dt * cy[s] * Yb[k] : 0.0);
            const double *Y = Ys + ((size_t)st * 4 + s) * per;
            orc_rhs_vjp(dim, n, kernel, sigma, tau, Y, Y + m, kb, kb + m, Yb, Yb + m);
            for (size_t k = 0; k < per; ++k) acc[k] += Yb[k];
        }
        memcpy(lam, acc, sizeof(double) * per);
    }
    memcpy(gq0, lam, sizeof(double) * m);
    memcpy(gp0, lam + m, sizeof(double) * m);
    free(Ys); free(y); free(ks); free(lam); free(acc); free(kb); free(Yb);
}

/* ---- Velocity field at arbitrary points (equation "u"):
 *   u(x) = sum_j G(|x - q_j|) p_j,   x given as m points, component-major (dim, m). ---- */
void orc_velocity(int dim, long n, long m, int kernel, double sigma,
                  const double *q, const double *p, const double *x, double *u)
{
#pragma omp parallel for schedule(static) if (m >= 256)
    for (long a = 0; a < m; ++a) {
        double v[3] = {0.0, 0.0, 0.0};
        for (long j = 0; j < n; ++j) {
            double s = 0.0;
            for (int c = 0; c < dim; ++c) {
                double d = x[c * m + a] - q[c * n + j];
                s += d * d;
            }
            double g = green(kernel, sigma, sqrt(s));
            for (int c = 0; c < dim; ++c) v[c] += g * p[c * n + j];
        }
        for (int c = 0; c < dim; ++c) u[c * m + a] = v[c];
    }
}

/* ---- Flow of arbitrary points along the geodesic: m passive points x carried by the
 * velocity field of equation "u" while the particles evolve by the N-particle system,
 *   dx_a/dt = sum_j G(|x_a - q_j|) p_j,
 * the whole state (q, p, x) advanced by the same classical RK4 steps as orc_shoot.  The
 * points do not act on the particles.  (The tau term of the inexact system moves only the
 * particles: the field of equation "u" has none.) --------------------------------------- */
void orc_flow_points(int dim, long n, long m, int kernel, double sigma, double tau, double T, int steps,
                     const double *q0, const double *p0, const double *x0,
                     double *q1, double *p1, double *x1)
{
    size_t mn = (size_t)dim * (size_t)n, mm = (size_t)dim * (size_t)m;
    double *q = (double *)malloc(sizeof(double) * mn), *p = (double *)malloc(sizeof(double) * mn);
    double *x = (double *)malloc(sizeof(double) * mm);
    double *qs = (double *)malloc(sizeof(double) * mn), *ps = (double *)malloc(sizeof(double) * mn);
    double *xs = (double *)malloc(sizeof(double) * mm);
    double *kq[4], *kp[4], *kx[4];
    for (int s = 0; s < 4; ++s) {
        kq[s] = (double *)malloc(sizeof(double) * mn);
        kp[s] = (double *)malloc(sizeof(double) * mn);
        kx[s] = (double *)malloc(sizeof(double) * mm);
    }
    memcpy(q, q0, sizeof(double) * mn);
    memcpy(p, p0, sizeof(double) * mn);
    memcpy(x, x0, sizeof(double) * mm);
    double dt = T / steps;
    const double cstage[4] = {0.0, 0.5, 0.5, 1.0};
    for (int step = 0; step < steps; ++step) {
        for (int s = 0; s < 4; ++s) {
            /* stage s: its input state (q, p, x) + c_s dt k_{s-1}; then k_s at that state */
            const double *qin = q, *pin = p, *xin = x;
            if (s > 0) {
                for (size_t k = 0; k < mn; ++k) {
                    qs[k] = q[k] + cstage[s] * dt * kq[s - 1][k];
                    ps[k] = p[k] + cstage[s] * dt * kp[s - 1][k];
                }
                for (size_t k = 0; k < mm; ++k) xs[k] = x[k] + cstage[s] * dt * kx[s - 1][k];
                qin = qs;
                pin = ps;
                xin = xs;
            }
            orc_rhs(dim, n, kernel, sigma, tau, qin, pin, kq[s], kp[s]);
            orc_velocity(dim, n, m, kernel, sigma, qin, pin, xin, kx[s]);
        }
        for (size_t k = 0; k < mn; ++k) {
            q[k] = q[k] + dt / 6.0 * (kq[0][k] + 2.0 * kq[1][k] + 2.0 * kq[2][k] + kq[3][k]);
            p[k] = p[k] + dt / 6.0 * (kp[0][k] + 2.0 * kp[1][k] + 2.0 * kp[2][k] + kp[3][k]);
        }
        for (size_t k = 0; k < mm; ++k)
            x[k] = x[k] + dt / 6.0 * (kx[0][k] + 2.0 * kx[1][k] + 2.0 * kx[2][k] + kx[3][k]);
    }
    memcpy(q1, q, sizeof(double) * mn);
    memcpy(p1, p, sizeof(double) * mn);
    memcpy(x1, x, sizeof(double) * mm);
    free(q); free(p); free(x); free(qs); free(ps); free(xs);
    for (int s = 0; s < 4; ++s) { free(kq[s]); free(kp[s]); free(kx[s]); }
}
