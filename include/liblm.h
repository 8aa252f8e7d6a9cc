/*
 * liblm.h -- C ABI of the MI355X (gfx950) library for geodesic landmark shooting with the
 * N-particle Euler-Poincare system (Camassa, Kuang & Lee, "A class of fast geodesic
 * shooting algorithms for template matching and its applications via the N-particle system
 * of the Euler-Poincare equations", arXiv 1510.03816).
 *
 * Problem statement (section "Algorithm for Landmark Shooting", equation "exact-matching"):
 * given labelled template landmarks X and target landmarks Y in R^dim, find initial momenta
 * p0 such that the flow of the N-particle system started at (X, p0) carries X onto Y at
 * t = 1.  Everything here runs on the GPU; no entry point falls back to host arithmetic.
 *
 * Conventions shared by every entry point
 *   - Arrays are DEVICE pointers unless a comment says "host".  Point sets are stored
 *     component-major ("SoA"): element (c, i) -- coordinate c of landmark i -- lives at
 *     x[c*n + i], c < dim, i < n.  Every array is contiguous and owned by the caller.
 *   - Element type of q/p/dq/dp/u buffers: double when params->dtype == LM_F64, float when
 *     LM_F32.  Feedback matching and the adjoint always take double buffers.
 *   - Kernels run on the caller's HIP stream (`stream`, a hipStream_t passed as void*;
 *     NULL = the default stream).  Entry points documented "asynchronous" return after
 *     enqueueing; those documented "synchronous" return after the stream has drained.
 *   - Temporary device memory is taken from the stream-ordered allocator of the stream's
 *     device and released on the same stream; nothing is cached between calls.
 *   - Arguments are checked before anything is enqueued: an invalid argument returns
 *     LM_EINVAL and enqueues nothing.  A HIP runtime failure returns LM_EHIP.
 *     lm_last_error() then describes the failure (thread-local text).
 *   - All entry points are thread-safe; calls that share output buffers must be ordered by
 *     the caller.
 */
#ifndef LIBLM_H
#define LIBLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lm_status {
    LM_OK = 0,
    LM_EINVAL = -1,        /* invalid argument (nothing was enqueued) */
    LM_ENOMEM = -2,        /* device memory exhausted */
    LM_EHIP = -3,          /* HIP runtime error (text in lm_last_error) */
    LM_ENOTCONV = -4,      /* iteration limit reached before the tolerance */
    LM_EDIVERGED = -5,     /* non-finite residual: the iteration blew up */
    LM_ESINGULAR = -6,     /* kernel matrix not numerically positive definite */
    LM_EUNSUPPORTED = -7   /* combination of options not provided */
} lm_status;

typedef enum lm_kernel {
    /* Conical kernel ("conon") G(r) = exp(-r/sigma): the Green's function of the
     * N-particle system for the metric H^{3/2} in the plane, normalised so that G(0) = 1
     * (equation of G_{1/2} and the normalisation stated with the exact-matching
     * experiments; sigma is the paper's alpha). */
    LM_KERNEL_CONON = 0,
    /* Gaussian kernel G(r) = exp(-r^2/sigma^2) (the smooth kernel of the metric H^infinity
     * in the metric-comparison section; sigma^2 is the paper's alpha^2). */
    LM_KERNEL_GAUSS = 1
} lm_kernel;

typedef enum lm_dtype { LM_F64 = 0, LM_F32 = 1 } lm_dtype;

/* How the K(X) solves of Algorithm 1 are done. */
typedef enum lm_solver {
    LM_SOLVE_AUTO = 0,    /* dense when its n x n factor fits in half the free device memory */
    LM_SOLVE_CG = 1,      /* matrix-free conjugate gradients: O(n) memory, K products on the fly */
    LM_SOLVE_DENSE = 2    /* Cholesky factor of K(X) + tau I built once (8 n^2 bytes), then two
                             triangular sweeps per solve */
} lm_solver;

/* Model parameters shared by every entry point. */
typedef struct lm_params {
    int32_t dim;      /* spatial dimension: 2 or 3 */
    int32_t kernel;   /* lm_kernel */
    int32_t dtype;    /* lm_dtype of q/p buffers (lm_rhs, lm_shoot, lm_hamiltonian, lm_velocity) */
    int32_t flags;    /* reserved, must be 0 */
    double sigma;     /* kernel width, > 0 and finite */
    double tau;       /* >= 0: weight of the inexact advection term tau*p_i (equation
                         "N-particle-inexact", where the paper writes sigma^2); 0 = exact */
    double cutoff;    /* 0 = every pair (exact).  > 0: tile skipping, an approximation that is
                         not in the paper.  Points are grouped in tiles of 64; a source tile
                         whose bounding box lies farther than `cutoff` from a target tile's box
                         is skipped, so only pairs farther apart than `cutoff` are dropped.
                         What a target loses is bounded by G(cutoff) sum_j |p_j| in velocity
                         and |G'(cutoff)| |p_i| sum_j |p_j| in force (for the Gaussian when
                         cutoff >= sigma/sqrt(2)).  lm_shoot and the feedback entry points
                         order the points by Morton code internally (outputs keep the
                         caller's order); lm_rhs and lm_velocity tile the caller's order, so
                         give them spatially ordered points.  lm_hamiltonian and lm_ksolve
                         ignore it and always sum every pair.  Needs n < 2^31. */
} lm_params;

/* Settings of Algorithm 1 (feedback-control iteration) with the constant gain M = h I. */
typedef struct lm_match_opts {
    double h;             /* search length h > 0 (M = h I) */
    double tol;           /* tolerance > 0 of the stopping test */
    int32_t max_iter;     /* >= 0: most momentum updates made */
    int32_t steps;        /* >= 1: RK4 steps of each shoot on t in [0, 1] */
    int32_t stop_rule;    /* 0: stop when max_{c,i} |Y - q(1)| < tol (exact matching);
                             1: stop when max |u^k - u^(k-1)| = h max|Y - q(1)|_(k-1) < tol
                                (the rule stated for inexact matching) */
    int32_t cg_max_iter;  /* conjugate-gradient iterations per solve; 0 = min(20n+100, 10000) */
    double cg_rtol;       /* relative residual of each K-solve; 0 = 1e-13 */
    double *resid_hist;   /* HOST, nullable: receives the residual of each shoot */
    int32_t hist_len;     /* capacity of resid_hist */
    int32_t solver;       /* K-solve: LM_SOLVE_AUTO, LM_SOLVE_CG or LM_SOLVE_DENSE */
    double f32_switch;    /* params->dtype = LM_F32 only.  0: every shoot in single precision.
                             > 0: single-precision shoots until a residual below f32_switch,
                             double-precision shoots after; the stopping test then accepts only
                             a double-precision residual (a single-precision one below tol is
                             re-shot in double precision before any further update).  A
                             single-precision residual not below 0.9 times the previous one
                             (the floor of single-precision shoots) also switches, re-shooting
                             those momenta in double precision */
} lm_match_opts;

/* What a feedback match reports (HOST struct).  GPU times come from HIP events on the
 * stream around each phase. */
typedef struct lm_match_info {
    int32_t iters;        /* momentum updates made before the final shoot */
    int32_t cg_iters;     /* conjugate-gradient iterations summed over every solve */
    double resid_inf;     /* max_{c,i} |Y - q(1)| of the final shoot */
    double H;             /* Hamiltonian 1/2 sum_ij (p_i.p_j) G(|X_i-X_j|) at (X, p0);
                             the values the paper prints are 2H */
    double shoot_ms;      /* GPU time of all shoots */
    double solve_ms;      /* GPU time of all K-solves and momentum updates */
    double factor_ms;     /* GPU time of the dense factorisation (0 with CG) */
    int32_t shoots;       /* shoots integrated: iters + 1, less one when p0 is zero (no landmark
                             then moves: the first shoot is the identity map, q(1) = X) */
} lm_match_info;

/* Right-hand side of the N-particle system (equation "N-particle"; with tau > 0 the inexact
 * system, equation "N-particle-inexact"):
 *     dq_i = sum_{j=1..n} G(|q_i - q_j|) p_j + tau p_i
 *     dp_i = -sum_{j != i} (p_i . p_j) G'(|q_i - q_j|) (q_i - q_j)/|q_i - q_j|
 * Distinct particles at the same point exert no force on each other.
 * q, p: inputs (dim, n); dq, dp: outputs (dim, n), must not overlap q or p.
 * Asynchronous. */
lm_status lm_rhs(const lm_params *params, int64_t n, const void *q, const void *p,
                 void *dq, void *dp, void *stream);

/* Launch plan of the pair sums of n points under `params` (host only: no GPU work, no
 * allocation): the kernel that lm_rhs and every RK4 stage of lm_shoot use, and its shape.
 * symmetric = 1: each unordered pair is evaluated once and serves both particles (double
 * precision from 128 tiles of 64 points on, single precision from 256; with tile skipping
 * from 768 in both); 0: the one-sided kernel, one target per lane.  The environment variable LM_SYM = 0 or 1 overrides that size rule and
 * LM_SYM_WAVES = 1, 2, 4 or 8 fixes the symmetric kernel's workgroup width (for tuning and
 * tests; both are read at every launch).  small = 1: shoots of this size (at most 128 points,
 * no cutoff) run whole inside one workgroup instead, of 4 or 8 waves by size (LM_SMALL = 0 or
 * 1 overrides the size rule, 1 allowing up to 256 points, and LM_SMALL_WAVES = 4, 8 or 16 fixes
 * the width, for tuning and tests).  LM_EINVAL on bad arguments. */
typedef struct lm_plan_info {
    int32_t symmetric;
    int32_t waves;           /* wavefronts per workgroup of the pair-sum launch */
    int64_t workgroups;      /* workgroups of the pair-sum launch */
    int32_t partial_slots;   /* partial sums per point added in a fixed order by a second
                                launch (1: the pair-sum launch finishes the sums itself) */
    int32_t small;
    int32_t rows;            /* symmetric: 64-point row tiles per wavefront (2, or 4 in the
                                widest tier); one-sided: 1 (one target per lane) */
} lm_plan_info;

lm_status lm_pair_plan(const lm_params *params, int64_t n, lm_plan_info *info);

/* Shooting map: integrates the N-particle system from (q0, p0) at t = 0 to t = t1 with
 * `steps` steps of the classical fourth-order Runge-Kutta method (the explicit integrator
 * the paper names for evolving the system in Algorithm 1, step 1).  Writes (q(t1), p(t1))
 * to q1, p1; q1/p1 may be the same buffers as q0/p0 (in-place shoot).  t1 may be any
 * finite value (t1 = 1 in Algorithm 1).  Asynchronous. */
lm_status lm_shoot(const lm_params *params, int64_t n, const void *q0, const void *p0,
                   double t1, int32_t steps, void *q1, void *p1, void *stream);

/* Discrete Hamiltonian H = 1/2 sum_i sum_j (p_i . p_j) G(|q_i - q_j|) (equation "H").
 * *H_out is a HOST double.  Synchronous. */
lm_status lm_hamiltonian(const lm_params *params, int64_t n, const void *q, const void *p,
                         double *H_out, void *stream);

/* Solves (K(X) + tau I) x = b for every component c, with K_ij = G(|X_i - X_j|): the
 * conversion of a velocity field u at the landmarks into momenta p (Algorithm 1, step 4,
 * read as p = K(X)^{-1} u).  solver: LM_SOLVE_CG (matrix-free conjugate gradients, stops when
 * ||b_c - K x_c||_2 <= rtol ||b_c||_2 for every c or after max_iter iterations), LM_SOLVE_DENSE
 * (Cholesky factor, rtol and max_iter unused; its triangular sweeps take one launch per
 * 128-row block, or, once the factor spans more than 8 blocks, three launches per 8 blocks
 * through stored inverses of the diagonal 1024 x 1024 parts, 7 x 128^2 more doubles per
 * block (1.4% of the factor at n = 65536); the
 * environment variable LM_DENSE_SUPER = 0/1 forces either form) or LM_SOLVE_AUTO.  X, b, x: double (dim, n);
 * x may alias b.  *iters_out (HOST, nullable) receives the CG iteration count (0 for dense).
 * cutoff is ignored: every pair enters K.  Synchronous.  LM_ESINGULAR if K is not
 * numerically positive definite (a CG curvature p.Kp <= 0 or a non-positive Cholesky
 * pivot); LM_ENOTCONV if CG reaches max_iter (x then holds the last iterate); LM_ENOMEM if
 * a forced dense factor does not fit. */
lm_status lm_ksolve(const lm_params *params, int64_t n, const double *X, const double *b,
                    double *x, double rtol, int32_t max_iter, int32_t solver, int32_t *iters_out,
                    void *stream);

/* Algorithm 1 (feedback-control iteration) with M = h I:
 *     p <- p0;  for k = 0, 1, ...:  q(1) = shoot(X, p);  e = Y - q(1);
 *         stop by opts->stop_rule;  u <- u + h e, i.e. p <- p + h (K(X) + tau I)^{-1} e
 * X, Y: double (dim, n).  p0: double (dim, n), in: initial momenta (zeros in the paper),
 * out: the final momenta.  q1 (nullable): double (dim, n), receives q(1) of the last
 * shoot.  info: HOST.  params->dtype = LM_F32 shoots in single precision while the
 * momenta, the residual and the K-solves stay in double; the dense factor's trailing updates
 * then multiply in single precision (the solves only steer the iteration; environment
 * LM_FACTOR_F32 = 0/1 overrides), staged from a float copy of each update's columns
 * (n x 1024 floats, counted in the dense solver's memory check; LM_FACTOR_F32_PANEL = 0
 * stages from the double matrix instead, with the same result).  opts->solver picks the
 * K-solve;
 * a dense factor is built once per call (K(X) is fixed during a match).  Synchronous.
 * Returns LM_OK, LM_ENOTCONV, LM_EDIVERGED (non-finite residual, as the paper's NaN for
 * h > 1) or LM_ESINGULAR; in every case p0 and info describe the last iterate. */
lm_status lm_feedback_match(const lm_params *params, const lm_match_opts *opts, int64_t n,
                            const double *X, const double *Y, double *p0, double *q1,
                            lm_match_info *info, void *stream);

/* What one feedback iteration reports (HOST struct). */
typedef struct lm_step_info {
    double resid_inf;     /* max_{c,i} |Y - q(1)| of this iteration's shoot */
    double shoot_ms;      /* GPU time of the shoot (HIP events on the stream) */
    double solve_ms;      /* GPU time of the K-solve and momentum update (0 if none) */
    int32_t converged;    /* 1 when resid_inf < tol (p then unchanged) */
    int32_t cg_iters;     /* CG iterations of the solve */
} lm_step_info;

/* One iteration of Algorithm 1 (the loop body of lm_feedback_match with the exact stopping
 * rule): shoots (X, p) to t = 1, computes r = max_{c,i} |Y - q(1)| and, unless r < tol,
 * updates p in place by p <- p + h (K(X) + tau I)^{-1} (Y - q(1)).  Lets a caller drive,
 * interleave, checkpoint or resume the iteration itself: its whole state is p.
 * opts->max_iter, stop_rule and the history fields are ignored.  q1 (nullable) receives
 * q(1).  info: HOST.  Synchronous.  LM_EDIVERGED for a non-finite residual. */
lm_status lm_feedback_step(const lm_params *params, const lm_match_opts *opts, int64_t n,
                           const double *X, const double *Y, double *p, double *q1,
                           lm_step_info *info, void *stream);

/* Reverse mode (not in the paper: it differentiates the inexact-matching energy of equation
 * "inexact-E" with respect to the initial momenta).  Double precision, cutoff = 0; other
 * settings return LM_EUNSUPPORTED.  Two distinct particles at the same point contribute only
 * the velocity-sum term, as in the forward sums. */

/* Vector-Jacobian product of the right-hand side at (q, p): (aq, ap) = J^T (a, b), where
 * (a, b) is a cotangent of (dq/dt, dp/dt).  All buffers double (dim, n); aq/ap must not
 * alias the inputs.  Asynchronous. */
lm_status lm_rhs_vjp(const lm_params *params, int64_t n, const double *q, const double *p,
                     const double *a, const double *b, double *aq, double *ap, void *stream);

/* Discrete adjoint of lm_shoot: (gq0, gp0) = J^T (gq1, gp1) for the RK4 map
 * (q0, p0) -> (q(t1), p(t1)) with `steps` steps.  The forward pass keeps the state every
 * ckpt_every steps (0 = keep every stage input of the whole shoot) and the reverse sweep
 * recomputes one segment at a time.  q1, p1 (nullable) receive the forward result.  gq0/gp0
 * may alias gq1/gp1.  All buffers double (dim, n).  Asynchronous. */
lm_status lm_shoot_adjoint(const lm_params *params, int64_t n, const double *q0, const double *p0,
                           double t1, int32_t steps, int32_t ckpt_every, const double *gq1,
                           const double *gp1, double *gq0, double *gp0, double *q1, double *p1,
                           void *stream);

/* Energy of inexact matching and its gradient in the initial momenta:
 *     E(p0) = reg/2 p0^T K(X) p0 + lam/2 |q(1) - Y|^2
 *     grad  = reg K(X) p0 + J^T (lam (q(1) - Y), 0)
 * With reg = 1 it is half the paper's inexact energy for lam = 1/sigma^2 (the geodesic's
 * kinetic energy written as 2H by eq. "E=2H"); reg = 0 leaves the least-squares shooting
 * objective, whose zero is an exact match.  q(1) is the RK4 shoot of (X, p0) over [0, 1];
 * *E_out is a HOST double; grad (dim, n) must not alias p0; q1 (nullable) receives q(1).
 * Synchronous. */
lm_status lm_energy_grad(const lm_params *params, int64_t n, const double *X, const double *Y,
                         const double *p0, double lam, double reg, int32_t steps, int32_t ckpt_every,
                         double *E_out, double *grad, double *q1, void *stream);

/* Settings and report of gradient-based matching (HOST structs). */
typedef struct lm_lbfgs_opts {
    double lam;           /* weight of the data term (>= 0) */
    double reg;           /* weight of the kinetic-energy regulariser (>= 0) */
    double gtol;          /* stop when max|grad| <= gtol * max|grad| at the start */
    double match_tol;     /* also stop when max|q(1) - Y| < match_tol (0 = off) */
    int32_t max_iter;     /* L-BFGS iterations */
    int32_t history;      /* stored (s, y) pairs, 0 = 8, at most 64 */
    int32_t steps;        /* RK4 steps per shoot */
    int32_t ckpt_every;   /* adjoint checkpoint spacing (0 = every stage kept) */
} lm_lbfgs_opts;

typedef struct lm_lbfgs_info {
    int32_t iters;        /* L-BFGS iterations made */
    int32_t evals;        /* energy-and-gradient evaluations (each a shoot and its adjoint) */
    double E;             /* final energy */
    double gnorm_inf;     /* final max |grad| */
    double resid_inf;     /* final max |q(1) - Y| */
} lm_lbfgs_info;

/* Gradient-based matching: minimises E(p0) of lm_energy_grad by limited-memory BFGS
 * (two-loop recursion, backtracking Armijo line search) from the momenta in p0, in place.
 * Every vector operation runs on the GPU; only scalars are read back.  It is the
 * gradient-descent counterpart of Algorithm 1's feedback iteration.  Synchronous.
 * LM_OK when a tolerance is met, LM_ENOTCONV after max_iter iterations or a failed line
 * search, LM_EDIVERGED on a non-finite energy; p0 and info describe the last iterate. */
lm_status lm_lbfgs_match(const lm_params *params, const lm_lbfgs_opts *opts, int64_t n,
                         const double *X, const double *Y, double *p0, lm_lbfgs_info *info,
                         void *stream);

/* Velocity field at arbitrary points (equation "u"): u(x_a) = sum_j G(|x_a - q_j|) p_j.
 * q, p: (dim, n); x, u: (dim, m).  Asynchronous. */
lm_status lm_velocity(const lm_params *params, int64_t n, const void *q, const void *p,
                      int64_t m, const void *x, void *u, void *stream);

/* Flow of arbitrary points along the geodesic (equation "u"; section "The prediction ability
 * of Algorithm 1"): shoots the particles (q0, p0) over [0, t1] with `steps` classical RK4 steps,
 * exactly as lm_shoot, and carries m passive points x along the velocity field of the moving
 * particles, dx_a/dt = u(x_a) = sum_j G(|x_a - q_j|) p_j, advanced by the same RK4 stages
 * (every stage evaluates u at the stage's points from the stage's particles).  The points do
 * not act on the particles; the tau term of the inexact system moves only the particles.
 * Warps grids or contours by the diffeomorphism the momenta generate, and continues a match
 * beyond its target (t1 > 1).  cutoff > 0 skips tiles of points farther than the radius from
 * a tile of particles (the bound of lm_params.cutoff applies to the velocity sums).
 * q0, p0: (dim, n); x0, x1: (dim, m), element type by params->dtype.  x1 receives x(t1) and may
 * be x0 itself; q1/p1 (nullable) receive q(t1), p(t1) and may be q0/p0 themselves.  x0/x1 must
 * not overlap the particle buffers.  Asynchronous. */
lm_status lm_flow_points(const lm_params *params, int64_t n, const void *q0, const void *p0, int64_t m,
                         const void *x0, double t1, int32_t steps, void *q1, void *p1, void *x1,
                         void *stream);

/* lm_shoot for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same shoot, with the same
 * kernels and results as lm_shoot, but its scratch memory (stage buffers, RK4 running sums,
 * the pair kernels' partial sums) comes from one fixed array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends; the call allocates and frees
 * nothing.  Every call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (other threads, other streams) race and corrupt each other's results, so the caller
 * must order them.  cutoff must be 0 (LM_EUNSUPPORTED otherwise).  A size whose scratch
 * exceeds the array -- 6 dim n element-size bytes plus the partial sums of the pair plan
 * (FP64 3-D: n = 16384 fits, n = 24576 does not) -- returns LM_ENOMEM with the bytes it
 * would need.
 * The stream must belong to the current device (LM_EINVAL otherwise).  Arguments and
 * aliasing as lm_shoot.  Asynchronous. */
lm_status lm_shoot_noalloc(const lm_params *params, int64_t n, const void *q0, const void *p0,
                           double t1, int32_t steps, void *q1, void *p1, void *stream);

/* ---------------------------------------------------------------------------------------
 * Batches of independent problems.  B problems of uneven size are concatenated in one
 * component-major array (dim, ntot), ntot = sum of the sizes: problem b owns columns
 * offs[b] .. offs[b+1]-1, and its particles interact only with each other (each problem is
 * the N-particle system of its own landmarks).  offs is a HOST array of B + 1 int64 values
 * with offs[0] = 0 and offs[b] < offs[b+1].  Every RK4 stage of every problem is one launch
 * over the whole batch: a work list of (problem, 64-target tile, source chunk) items sorted
 * by cost, walked by a persistent grid.  cutoff must be 0.
 * --------------------------------------------------------------------------------------- */
#define LM_BATCH_BUCKETS 4

/* Launch shape of a batch (HOST struct).  Problems fall into size buckets; bucket k holds
 * the problems with bucket_max[k-1] < N_b <= bucket_max[k] (bucket_max[-1] = 0). */
typedef struct lm_batch_tuning {
    int64_t bucket_max[LM_BATCH_BUCKETS]; /* ascending; the last >= every N_b */
    int32_t split[LM_BATCH_BUCKETS];      /* source chunks per 64-target tile, 1..64
                                             (1: the item owns all its sources) */
    int32_t groups;                       /* persistent grid in workgroups of 4 waves;
                                             0 = one wave per work item */
    int32_t graph_steps;                  /* RK4 steps per captured hipGraph in a shoot;
                                             0 = every kernel launched directly */
    int32_t sym_min;                      /* problems of at least sym_min points evaluate
                                             each unordered pair once (the symmetric
                                             kernel, one superblock pair per workgroup);
                                             0 = never */
    int32_t sym_waves;                    /* its wavefronts per workgroup: 1, 2, 4 or 8 */
    double stage_us;                      /* written by lm_batch_autotune: measured time of
                                             one stage with this shape (microseconds) */
} lm_batch_tuning;

/* A launch shape that needs no measurement (HOST only, no GPU call).  Validates offs. */
lm_status lm_batch_default_tuning(int32_t B, const int64_t *offs, lm_batch_tuning *out);

/* Autotuner: times candidate launch shapes on this batch (right-hand-side evaluations at
 * (q, p), dim x ntot device arrays of params->dtype, and short graph-replayed shoots) with
 * HIP events, one parameter at a time from the default (grid size, then each occupied
 * bucket's source split, then the symmetric threshold and width, then the
 * steps per graph), and writes the fastest to *out.
 * Synchronous; q and p are not modified. */
lm_status lm_batch_autotune(const lm_params *params, int32_t B, const int64_t *offs,
                            const void *q, const void *p, lm_batch_tuning *out, void *stream);

/* lm_rhs for every problem of a batch.  tuning: nullable (NULL = the default shape).
 * Asynchronous. */
lm_status lm_rhs_batched(const lm_params *params, int32_t B, const int64_t *offs,
                         const void *q, const void *p, void *dq, void *dp,
                         const lm_batch_tuning *tuning, void *stream);

/* lm_shoot for every problem of a batch (the same t1 and steps for all).  With
 * tuning->graph_steps > 0 the RK4 steps are captured once into a hipGraph and replayed;
 * the call then returns after the shoot has finished.  Otherwise asynchronous. */
lm_status lm_shoot_batched(const lm_params *params, int32_t B, const int64_t *offs,
                           const void *q0, const void *p0, double t1, int32_t steps,
                           void *q1, void *p1, const lm_batch_tuning *tuning, void *stream);

/* Algorithm 1 for every problem of a batch, all problems iterating together: one batched
 * shoot per iteration, then for every problem not yet stopped the residual test and the
 * update p <- p + h (K(X_b) + tau I)^{-1} (Y_b - q_b(1)) with the dense factor of its own
 * kernel matrix.  A problem stops when its residual passes (stop_rule 0 only), diverges or
 * has a singular K; the batch runs until every problem has stopped or max_iter updates.
 * params->dtype = LM_F32 shoots in single precision from FP64 master momenta; residuals,
 * solves and updates are FP64.  X, Y, p0 (in: guess, out: result), q1 (nullable): FP64
 * (dim, ntot) device arrays.  info, status: HOST arrays of B entries (per-problem iteration
 * count, final residual, H at (X, p0), status); the *_ms fields of every entry hold the
 * batch totals.  Returns LM_OK when every problem converged, else the first of
 * LM_EDIVERGED, LM_ESINGULAR, LM_ENOTCONV that some problem ended with.  tuning: nullable
 * (NULL = the default shape); when the problems still running would launch fewer than two
 * waves per SIMD, a shoot narrows the symmetric superblocks and splits the one-sided sources
 * further (environment LM_BATCH_FILL: waves per SIMD, 0 = keep the tuning's shape).  The
 * solves of problems above 1024 points run across many workgroups per problem, the rest with
 * one workgroup each (environment LM_BATCH_WIDE_MIN: the size threshold).  Synchronous. */
lm_status lm_feedback_match_batched(const lm_params *params, const lm_match_opts *opts, int32_t B,
                                    const int64_t *offs, const double *X, const double *Y,
                                    double *p0, double *q1, lm_match_info *info, int32_t *status,
                                    const lm_batch_tuning *tuning, void *stream);

/* Text describing the last non-OK status returned on the calling thread ("" if none). */
const char *lm_last_error(void);

/* Library version string. */
const char *lm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBLM_H */
