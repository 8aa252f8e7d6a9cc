/*
 * abi_check.c -- TEST INFRASTRUCTURE.  Drives the host side of the C ABI (include/liblm.h)
 * under the host sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer) without a GPU:
 * every call here is answered by host code before anything is enqueued -- argument
 * validation (each entry point with invalid parameters, sizes, pointers, aliasing and
 * options) and the host-only planners (lm_pair_plan over the size rules, and
 * lm_batch_default_tuning over valid and invalid batch layouts).  Device addresses are
 * fake and never dereferenced.  Exit status 0 when every status is the one expected.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "liblm.h"

static int g_bad = 0;

static void expect(const char *what, lm_status got, lm_status want)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, lm_last_error());
        g_bad = 1;
    } else if (want != LM_OK && strlen(lm_last_error()) == 0) {
        fprintf(stderr, "%s: no error text\n", what);
        g_bad = 1;
    }
}

static lm_params params(int dim, int kernel, int dtype, double sigma, double tau, double cutoff)
{
    lm_params p;
    memset(&p, 0, sizeof p);
    p.dim = dim;
    p.kernel = kernel;
    p.dtype = dtype;
    p.sigma = sigma;
    p.tau = tau;
    p.cutoff = cutoff;
    return p;
}

#define FAKE(a) ((void *)(uintptr_t)(a))

int main(void)
{
    void *q = FAKE(0x100000), *p = FAKE(0x200000), *o1 = FAKE(0x300000), *o2 = FAKE(0x400000);
    void *x = FAKE(0x500000);
    lm_params ok = params(2, 0, 0, 0.5, 0.0, 0.0);

    /* parameter validation, through lm_rhs */
    lm_params bad[] = {params(4, 0, 0, 0.5, 0, 0), params(2, 7, 0, 0.5, 0, 0), params(2, 0, 3, 0.5, 0, 0),
                       params(2, 0, 0, 0.0, 0, 0), params(2, 0, 0, NAN, 0, 0), params(2, 0, 0, INFINITY, 0, 0),
                       params(2, 0, 0, 0.5, -1.0, 0), params(2, 0, 0, 0.5, 0, -1.0), params(2, 0, 0, 0.5, NAN, 0)};
    for (size_t k = 0; k < sizeof bad / sizeof bad[0]; ++k) expect("lm_rhs bad params", lm_rhs(&bad[k], 10, q, p, o1, o2, NULL), LM_EINVAL);
    lm_params flags = ok;
    flags.flags = 1;
    expect("lm_rhs flags", lm_rhs(&flags, 10, q, p, o1, o2, NULL), LM_EINVAL);
    expect("lm_rhs NULL params", lm_rhs(NULL, 10, q, p, o1, o2, NULL), LM_EINVAL);
    expect("lm_rhs n = 0", lm_rhs(&ok, 0, q, p, o1, o2, NULL), LM_EINVAL);
    expect("lm_rhs n too large", lm_rhs(&ok, ((int64_t)1 << 40), q, p, o1, o2, NULL), LM_EINVAL);
    expect("lm_rhs NULL q", lm_rhs(&ok, 10, NULL, p, o1, o2, NULL), LM_EINVAL);
    expect("lm_rhs dq aliasing q", lm_rhs(&ok, 10, q, p, q, o2, NULL), LM_EINVAL);

    /* shoots */
    expect("lm_shoot steps 0", lm_shoot(&ok, 10, q, p, 1.0, 0, o1, o2, NULL), LM_EINVAL);
    expect("lm_shoot t1 inf", lm_shoot(&ok, 10, q, p, INFINITY, 5, o1, o2, NULL), LM_EINVAL);
    expect("lm_shoot q1 == p1", lm_shoot(&ok, 10, q, p, 1.0, 5, o1, o1, NULL), LM_EINVAL);
    expect("lm_shoot NULL p1", lm_shoot(&ok, 10, q, p, 1.0, 5, o1, NULL, NULL), LM_EINVAL);
    expect("lm_flow_points steps 0", lm_flow_points(&ok, 10, q, p, 5, x, 1.0, 0, NULL, NULL, x, NULL), LM_EINVAL);
    expect("lm_flow_points m 0", lm_flow_points(&ok, 10, q, p, 0, x, 1.0, 5, NULL, NULL, x, NULL), LM_EINVAL);
    expect("lm_flow_points x1 in q0", lm_flow_points(&ok, 10, q, p, 5, x, 1.0, 5, NULL, NULL, FAKE(0x100008), NULL),
           LM_EINVAL);
    expect("lm_flow_points NULL x1", lm_flow_points(&ok, 10, q, p, 5, x, 1.0, 5, NULL, NULL, NULL, NULL), LM_EINVAL);
    expect("lm_velocity m 0", lm_velocity(&ok, 10, q, p, 0, x, o1, NULL), LM_EINVAL);
    expect("lm_velocity NULL u", lm_velocity(&ok, 10, q, p, 5, x, NULL, NULL), LM_EINVAL);
    double H = 0.0;
    expect("lm_hamiltonian NULL H", lm_hamiltonian(&ok, 10, q, p, NULL, NULL), LM_EINVAL);
    expect("lm_hamiltonian n 0", lm_hamiltonian(&ok, 0, q, p, &H, NULL), LM_EINVAL);

    /* K-solve and Algorithm 1 */
    expect("lm_ksolve bad solver", lm_ksolve(&ok, 10, q, p, o1, 1e-12, 0, 9, NULL, NULL), LM_EINVAL);
    expect("lm_ksolve NULL x", lm_ksolve(&ok, 10, q, p, NULL, 1e-12, 0, 0, NULL, NULL), LM_EINVAL);
    lm_match_opts mo;
    memset(&mo, 0, sizeof mo);
    mo.h = 0.8;
    mo.tol = 1e-6;
    mo.max_iter = 10;
    mo.steps = 10;
    lm_match_info info;
    lm_match_opts m2 = mo;
    m2.h = 0.0;
    expect("lm_feedback_match h 0", lm_feedback_match(&ok, &m2, 10, q, p, o1, NULL, &info, NULL), LM_EINVAL);
    m2 = mo;
    m2.tol = -1.0;
    expect("lm_feedback_match tol < 0", lm_feedback_match(&ok, &m2, 10, q, p, o1, NULL, &info, NULL), LM_EINVAL);
    m2 = mo;
    m2.steps = 0;
    expect("lm_feedback_match steps 0", lm_feedback_match(&ok, &m2, 10, q, p, o1, NULL, &info, NULL), LM_EINVAL);
    m2 = mo;
    m2.stop_rule = 5;
    expect("lm_feedback_match stop rule", lm_feedback_match(&ok, &m2, 10, q, p, o1, NULL, &info, NULL), LM_EINVAL);
    expect("lm_feedback_match NULL info", lm_feedback_match(&ok, &mo, 10, q, p, o1, NULL, NULL, NULL), LM_EINVAL);
    expect("lm_feedback_match NULL opts", lm_feedback_match(&ok, NULL, 10, q, p, o1, NULL, &info, NULL), LM_EINVAL);
    lm_step_info si;
    m2 = mo;
    m2.h = -1.0;
    expect("lm_feedback_step h < 0", lm_feedback_step(&ok, &m2, 10, q, p, o1, NULL, &si, NULL), LM_EINVAL);

    /* reverse mode: double precision and every pair only */
    lm_params f32 = params(3, 1, 1, 0.3, 0.0, 0.0), cut = params(3, 1, 0, 0.3, 0.0, 0.5);
    expect("lm_rhs_vjp f32", lm_rhs_vjp(&f32, 10, q, p, o1, o2, x, FAKE(0x600000), NULL), LM_EUNSUPPORTED);
    expect("lm_rhs_vjp cutoff", lm_rhs_vjp(&cut, 10, q, p, o1, o2, x, FAKE(0x600000), NULL), LM_EUNSUPPORTED);
    expect("lm_shoot_adjoint steps 0",
           lm_shoot_adjoint(&ok, 10, q, p, 1.0, 0, 0, o1, o2, x, FAKE(0x600000), NULL, NULL, NULL), LM_EINVAL);
    double E = 0.0;
    expect("lm_energy_grad lam < 0", lm_energy_grad(&ok, 10, q, p, o1, -1.0, 1.0, 10, 0, &E, o2, NULL, NULL),
           LM_EINVAL);
    lm_lbfgs_opts lo;
    memset(&lo, 0, sizeof lo);
    lo.lam = 1.0;
    lo.reg = 1.0;
    lo.max_iter = 10;
    lo.steps = 0;
    lm_lbfgs_info li;
    expect("lm_lbfgs_match steps 0", lm_lbfgs_match(&ok, &lo, 10, q, p, o1, &li, NULL), LM_EINVAL);
    lo.steps = 10;
    lo.history = 100;
    expect("lm_lbfgs_match history", lm_lbfgs_match(&ok, &lo, 10, q, p, o1, &li, NULL), LM_EINVAL);

    /* the planners (host only): every size class, both precisions, with and without cutoff */
    const int64_t ns[] = {1, 2, 63, 64, 65, 256, 257, 4096, 5120, 8191, 8192, 12288, 49152, 65536, 131072,
                          (int64_t)1 << 20, (int64_t)1 << 24};
    for (int dt = 0; dt <= 1; ++dt)
        for (int dim = 2; dim <= 3; ++dim)
            for (int c = 0; c <= 1; ++c)
                for (size_t k = 0; k < sizeof ns / sizeof ns[0]; ++k) {
                    lm_params pp = params(dim, 0, dt, 0.1, 0.0, c ? 0.3 : 0.0);
                    lm_plan_info pi;
                    expect("lm_pair_plan", lm_pair_plan(&pp, ns[k], &pi), LM_OK);
                    if (pi.workgroups < 1 || pi.waves < 1 || pi.partial_slots < 1) {
                        fprintf(stderr, "lm_pair_plan n=%lld: empty plan\n", (long long)ns[k]);
                        g_bad = 1;
                    }
                }
    lm_plan_info pi;
    expect("lm_pair_plan n 0", lm_pair_plan(&ok, 0, &pi), LM_EINVAL);
    expect("lm_pair_plan NULL info", lm_pair_plan(&ok, 10, NULL), LM_EINVAL);

    lm_batch_tuning bt;
    int64_t offs1[] = {0, 33, 100, 4196, 4200, 8000};
    expect("lm_batch_default_tuning", lm_batch_default_tuning(5, offs1, &bt), LM_OK);
    int64_t offs2[] = {0, 1};
    expect("lm_batch_default_tuning one point", lm_batch_default_tuning(1, offs2, &bt), LM_OK);
    int64_t offs3[] = {0, 10, 10, 20};
    expect("lm_batch_default_tuning empty problem", lm_batch_default_tuning(3, offs3, &bt), LM_EINVAL);
    int64_t offs4[] = {5, 10};
    expect("lm_batch_default_tuning offs[0] != 0", lm_batch_default_tuning(1, offs4, &bt), LM_EINVAL);
    expect("lm_batch_default_tuning B 0", lm_batch_default_tuning(0, offs1, &bt), LM_EINVAL);
    expect("lm_batch_default_tuning NULL offs", lm_batch_default_tuning(3, NULL, &bt), LM_EINVAL);
    expect("lm_shoot_batched steps 0", lm_shoot_batched(&ok, 5, offs1, q, p, 1.0, 0, o1, o2, NULL, NULL), LM_EINVAL);
    expect("lm_rhs_batched bad offs", lm_rhs_batched(&ok, 3, offs3, q, p, o1, o2, NULL, NULL), LM_EINVAL);
    expect("lm_rhs_batched cutoff", lm_rhs_batched(&cut, 5, offs1, q, p, o1, o2, NULL, NULL), LM_EUNSUPPORTED);

    if (strlen(lm_version()) == 0) g_bad = 1;
    if (g_bad) return 1;
    printf("C ABI host-side sanitizer run: ok\n");
    return 0;
}
