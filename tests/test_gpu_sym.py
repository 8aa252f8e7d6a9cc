"""The symmetric pair kernel (each unordered pair evaluated once) against the FP64 oracle
and against the one-sided kernel, through the C ABI (needs an MI355X).

LM_SYM=1 forces the symmetric kernel at any size and LM_SYM_WAVES fixes its workgroup
width, so every width and ragged superblocks are covered at sizes the oracle finishes in
seconds; the size rule alone picks it from N = 8192 on.
"""

import os

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1510_03816_amd as lm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


class _env:
    """Sets LM_SYM / LM_SYM_WAVES / LM_SYM_ROWS for the duration of a block."""

    def __init__(self, **kv):
        self.kv = {k: str(v) for k, v in kv.items()}

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


TOL = {lm.F64: 1e-10, lm.F32: 1e-4}


def dev(a, dtype=lm.F64):
    tdt = torch.float64 if dtype == lm.F64 else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=tdt, device=DEV)


def host(t):
    return t.detach().double().cpu().numpy()


def rounded(a, dtype):
    return a.astype(np.float32).astype(np.float64) if dtype == lm.F32 else a


def rel_err(got, want):
    scale = np.max(np.abs(want))
    d = np.max(np.abs(got - want))
    return d / scale if scale > 0 else d


def gpu_rhs(q, p, kernel, sigma, tau=0.0, dtype=lm.F64):
    prm = lm.make_params(q.shape[0], kernel, sigma, tau=tau, dtype=dtype)
    qd, pd = dev(q, dtype), dev(p, dtype)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    lm.lm_rhs(prm, qd, pd, dq, dp)
    torch.cuda.synchronize()
    return host(dq), host(dp)


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 2, 64, 65, 700, 3007])
def test_sym_rhs_matches_oracle(n, dim, kernel, waves, dtype):
    q, p = inputs.random_state(n, dim, seed=[110, n, dim], box=1.0, pscale=0.3)
    q, p = rounded(q, dtype), rounded(p, dtype)
    sigma, tau = (0.3 if dim == 3 else 0.25), 0.1
    dq_o, dp_o = oracle.rhs(q, p, kernel, sigma, tau)
    print("sym rhs n=%d dim=%d kernel=%d waves=%d dtype=%d" % (n, dim, kernel, waves, dtype), flush=True)
    with _env(LM_SYM=1, LM_SYM_WAVES=waves):
        dq, dp = gpu_rhs(q, p, kernel, sigma, tau, dtype)
    eq, ep = rel_err(dq, dq_o), rel_err(dp, dp_o)
    print("  %.2e %.2e" % (eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]
    if n == 1:
        assert np.all(dp == 0.0)


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 65, 700, 3007])
def test_sym_wide_rows_match_oracle(n, dim, kernel, waves, dtype):
    """Four row tiles per wave (the widest tier's kernel), forced at small sizes: the sums
    with forces run it, the velocity-only K x of a CG solve falls back to two rows."""
    q, p = inputs.random_state(n, dim, seed=[120, n, dim], box=1.0, pscale=0.3)
    q, p = rounded(q, dtype), rounded(p, dtype)
    sigma, tau = (0.3 if dim == 3 else 0.25), 0.1
    dq_o, dp_o = oracle.rhs(q, p, kernel, sigma, tau)
    print("sym wide rhs n=%d dim=%d kernel=%d waves=%d dtype=%d" % (n, dim, kernel, waves, dtype), flush=True)
    with _env(LM_SYM=1, LM_SYM_WAVES=waves, LM_SYM_ROWS=4):
        dq, dp = gpu_rhs(q, p, kernel, sigma, tau, dtype)
    assert rel_err(dq, dq_o) <= TOL[dtype] and rel_err(dp, dp_o) <= TOL[dtype]


def test_sym_wide_rows_shoot_and_velocity_only_products():
    pr = inputs.config_curve2d(1000)
    oq, op = oracle.shoot(pr.X, pr.p_bench(), pr.kernel, pr.sigma, 10)
    X = pr.X
    b = np.random.default_rng(121).standard_normal(X.shape)
    st, L = oracle.cholesky(oracle.kmatrix(X, pr.kernel, pr.sigma))
    want = np.stack([oracle.cholesky_solve(L, b[c]) for c in range(2)])
    prm = lm.make_params(2, pr.kernel, pr.sigma)
    with _env(LM_SYM=1, LM_SYM_WAVES=4, LM_SYM_ROWS=4):
        q, p = dev(pr.X), dev(pr.p_bench())
        q1, p1 = torch.empty_like(q), torch.empty_like(p)
        lm.lm_shoot(prm, q, p, 1.0, 10, q1, p1)
        x = torch.empty_like(q)
        lm.lm_ksolve(prm, dev(X), dev(b), x, rtol=1e-13, solver=lm.SOLVE_CG)
        torch.cuda.synchronize()
    assert rel_err(host(q1), oq) <= 1e-10 and rel_err(host(p1), op) <= 1e-10
    assert rel_err(host(x), want) <= 1e-8


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_coincident_particles(kernel):
    q, p = inputs.random_state(300, 3, seed=111)
    q[:, 100:140] = q[:, 0:40]            # coincident distinct particles, across tiles
    q[:, 200] = q[:, 201]
    dq_o, dp_o = oracle.rhs(q, p, kernel, 0.4)
    with _env(LM_SYM=1, LM_SYM_WAVES=2):
        dq, dp = gpu_rhs(q, p, kernel, 0.4)
    assert np.all(np.isfinite(dp))
    assert rel_err(dq, dq_o) <= 1e-10 and rel_err(dp, dp_o) <= 1e-10


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_agrees_with_one_sided_kernel(kernel):
    """Both kernels on the same input; they differ only in summation order."""
    q, p = inputs.random_state(5000, 3, seed=112, pscale=0.3)
    with _env(LM_SYM=0):
        a = gpu_rhs(q, p, kernel, 0.2)
    with _env(LM_SYM=1, LM_SYM_WAVES=4):
        b = gpu_rhs(q, p, kernel, 0.2)
    assert rel_err(b[0], a[0]) <= 1e-13 and rel_err(b[1], a[1]) <= 1e-13


@pytest.mark.parametrize("n,dtype,waves", [(12289, lm.F64, 2), (30000, lm.F64, 2), (17000, lm.F32, 1),
                                           (33000, lm.F32, 2)])
def test_sym_by_size_rule_sampled(n, dtype, waves):
    """Sizes where the size rule itself picks the symmetric kernel (one or two waves per
    workgroup; four are covered at N = 65536 by the full-size tests); sampled rows against the
    oracle, and the forces sum to zero: in FP64 within 1e-9 of the largest force, in FP32 within
    1e-6 of the sum of the forces' magnitudes (the rows' and the columns' float sums round the
    same pair terms in different orders; measured 4.6e-8 at N = 17000)."""
    pr = inputs.config_sphere3d(n)
    q, p = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    plan = lm.lm_pair_plan(lm.make_params(3, pr.kernel, pr.sigma, dtype=dtype), n)
    assert plan["symmetric"] == 1 and plan["waves"] == waves
    dq, dp = gpu_rhs(q, p, pr.kernel, pr.sigma, dtype=dtype)
    idx = np.sort(np.random.default_rng(113).choice(n, 128, replace=False))
    idx = np.concatenate([[0, 63, 64, 127, 128, n - 1], idx])
    rq, rp = oracle.rhs_rows(q, p, idx, pr.kernel, pr.sigma)
    assert rel_err(dq[:, idx], rq) <= TOL[dtype] and rel_err(dp[:, idx], rp) <= TOL[dtype]
    if dtype == lm.F64:
        assert np.max(np.abs(dp.sum(axis=1))) <= 1e-9 * np.max(np.abs(dp))
    else:
        assert np.all(np.abs(dp.sum(axis=1)) <= 1e-6 * np.abs(dp).sum(axis=1))


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_sym_shoot_matches_oracle_and_is_deterministic(dtype):
    pr = inputs.config_curve2d(700)
    X, P = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    oq, op = oracle.shoot(X, P, pr.kernel, pr.sigma, 40)
    prm = lm.make_params(2, pr.kernel, pr.sigma, dtype=dtype)
    outs = []
    with _env(LM_SYM=1, LM_SYM_WAVES=2):
        for _ in range(2):
            q, p = dev(X, dtype), dev(P, dtype)
            q1, p1 = torch.empty_like(q), torch.empty_like(p)
            lm.lm_shoot(prm, q, p, 1.0, 40, q1, p1)
            torch.cuda.synchronize()
            outs.append((host(q1), host(p1)))
    assert rel_err(outs[0][0], oq) <= TOL[dtype] and rel_err(outs[0][1], op) <= TOL[dtype]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_sym_cg_ksolve_matches_cholesky():
    """The CG solver's products K x run through the velocity-only symmetric kernel."""
    pr = inputs.config_curve2d(1000)
    X = pr.X
    b = np.random.default_rng(114).standard_normal(X.shape)
    st, L = oracle.cholesky(oracle.kmatrix(X, pr.kernel, pr.sigma))
    assert st == 0
    want = np.stack([oracle.cholesky_solve(L, b[c]) for c in range(X.shape[0])])
    prm = lm.make_params(X.shape[0], pr.kernel, pr.sigma)
    x = torch.empty((X.shape[0], X.shape[1]), dtype=torch.float64, device=DEV)
    with _env(LM_SYM=1, LM_SYM_WAVES=4):
        it = lm.lm_ksolve(prm, dev(X), dev(b), x, rtol=1e-13, solver=lm.SOLVE_CG)
    print("%d CG iterations, rel err %.2e" % (it, rel_err(host(x), want)))
    assert rel_err(host(x), want) <= 1e-8


# ------------------------------------------------------------------ reverse mode


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 65, 700, 3007])
def test_sym_vjp_matches_oracle(n, dim, kernel, waves):
    q, p = inputs.random_state(n, dim, seed=[115, n, dim], pscale=0.3)
    rng = np.random.default_rng([116, n])
    a, b = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
    q[:, n // 2] = q[:, 0]                 # a coincident pair (for n > 2)
    prm = lm.make_params(dim, kernel, 0.3, tau=0.2)
    aq, ap = torch.empty((dim, n), dtype=torch.float64, device=DEV), torch.empty((dim, n), dtype=torch.float64, device=DEV)
    print("sym vjp n=%d dim=%d kernel=%d waves=%d" % (n, dim, kernel, waves), flush=True)
    with _env(LM_SYM=1, LM_SYM_WAVES=waves):
        lm.lm_rhs_vjp(prm, dev(q), dev(p), dev(a), dev(b), aq, ap)
        torch.cuda.synchronize()
    oq, op = oracle.rhs_vjp(q, p, a, b, kernel, 0.3, 0.2)
    eq, ep = rel_err(host(aq), oq), rel_err(host(ap), op)
    print("  %.2e %.2e" % (eq, ep))
    assert eq <= 1e-10 and ep <= 1e-10


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_vjp_agrees_with_one_sided_kernel(kernel):
    q, p = inputs.random_state(6000, 3, seed=117, pscale=0.3)
    rng = np.random.default_rng(118)
    a, b = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
    prm = lm.make_params(3, kernel, 0.2)
    out = []
    for env in ({"LM_SYM": 0}, {"LM_SYM": 1, "LM_SYM_WAVES": 4}):
        aq, ap = torch.empty((3, 6000), dtype=torch.float64, device=DEV), torch.empty((3, 6000), dtype=torch.float64, device=DEV)
        with _env(**env):
            lm.lm_rhs_vjp(prm, dev(q), dev(p), dev(a), dev(b), aq, ap)
            torch.cuda.synchronize()
        out.append((host(aq), host(ap)))
    assert rel_err(out[1][0], out[0][0]) <= 1e-13 and rel_err(out[1][1], out[0][1]) <= 1e-13


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_shoot_adjoint_and_energy_gradient_match_oracle(kernel):
    """Forward stages and VJP stages both symmetric (forced), through the checkpointed adjoint."""
    pr = inputs.config_sphere3d(500, kernel=kernel, sigma=0.2)
    q0, p0 = pr.X, 0.3 * pr.p_bench()
    rng = np.random.default_rng(119)
    gq1, gp1 = rng.standard_normal(q0.shape), rng.standard_normal(q0.shape)
    oq, op = oracle.shoot_adjoint(q0, p0, gq1, gp1, kernel, pr.sigma, 10, T=0.8, tau=0.1)
    E_o, g_o = oracle.energy_and_grad(pr.X, pr.Y, p0, kernel, pr.sigma, 100.0, 10)
    with _env(LM_SYM=1, LM_SYM_WAVES=2):
        prm = lm.make_params(3, kernel, pr.sigma, tau=0.1)
        gq0, gp0 = torch.empty((3, 500), dtype=torch.float64, device=DEV), torch.empty((3, 500), dtype=torch.float64, device=DEV)
        lm.lm_shoot_adjoint(prm, dev(q0), dev(p0), 0.8, 10, 3, dev(gq1), dev(gp1), gq0, gp0)
        prm0 = lm.make_params(3, kernel, pr.sigma)
        g = torch.empty((3, 500), dtype=torch.float64, device=DEV)
        E = lm.lm_energy_grad(prm0, dev(pr.X), dev(pr.Y), dev(p0), 100.0, 10, g, ckpt_every=3)
        torch.cuda.synchronize()
    assert rel_err(host(gq0), oq) <= 1e-10 and rel_err(host(gp0), op) <= 1e-10
    assert E == pytest.approx(E_o, rel=1e-11)
    assert rel_err(host(g), g_o) <= 1e-10


# ------------------------------------------------------------------ tile skipping


def _morton_sorted(X):
    lo, hi = X.min(axis=1, keepdims=True), X.max(axis=1, keepdims=True)
    g = np.clip(((X - lo) / (hi - lo) * 1023).astype(np.int64), 0, 1023)
    key = np.zeros(X.shape[1], dtype=np.int64)
    for b in range(10):
        for c in range(X.shape[0]):
            key |= ((g[c] >> b) & 1) << (X.shape[0] * b + c)
    return np.argsort(key, kind="stable")


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_cutoff_at_negligible_radius_meets_exact_parity(kernel, waves, dtype):
    pr = inputs.config_sphere3d(6000, kernel=kernel, sigma=0.05)
    perm = _morton_sorted(pr.X)
    q, p = rounded(pr.X[:, perm], dtype), rounded(pr.p_bench()[:, perm], dtype)
    rc = pr.sigma * (36.9 if kernel == 0 else 36.9 ** 0.5)
    dq_o, dp_o = oracle.rhs(q, p, kernel, pr.sigma)
    prm = lm.make_params(3, kernel, pr.sigma, cutoff=rc, dtype=dtype)
    qd, pd = dev(q, dtype), dev(p, dtype)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    with _env(LM_SYM=1, LM_SYM_WAVES=waves):
        lm.lm_rhs(prm, qd, pd, dq, dp)
        torch.cuda.synchronize()
    assert rel_err(host(dq), dq_o) <= TOL[dtype] and rel_err(host(dp), dp_o) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_sym_cutoff_error_within_certified_bound_and_matches_one_sided(kernel, dtype):
    """At a radius that drops pairs, the symmetric kernel skips exactly the tile pairs the
    one-sided kernel skips: the same pairs are dropped, so both stay within the certified
    bound and agree to rounding (single precision: the bound's slack is 1e-5 of the largest
    value, and the two kernels, which round in different orders, agree within the FP32 parity
    bar; the Gaussian's forces cancel, so their rounding reaches 2e-5 of the largest force)."""
    pr = inputs.config_sphere3d(8000, kernel=kernel, sigma=0.05)
    perm = _morton_sorted(pr.X)
    q, p = rounded(pr.X[:, perm], dtype), rounded(pr.p_bench()[:, perm], dtype)
    rc = 3.0 * pr.sigma
    dq_o, dp_o = oracle.rhs(q, p, kernel, pr.sigma)
    prm = lm.make_params(3, kernel, pr.sigma, cutoff=rc, dtype=dtype)
    out = []
    for env in ({"LM_SYM": 0}, {"LM_SYM": 1, "LM_SYM_WAVES": 2}):
        qd, pd = dev(q, dtype), dev(p, dtype)
        dq, dp = torch.empty_like(qd), torch.empty_like(pd)
        with _env(**env):
            lm.lm_rhs(prm, qd, pd, dq, dp)
            torch.cuda.synchronize()
        out.append((host(dq), host(dp)))
    G = np.exp(-rc / pr.sigma) if kernel == 0 else np.exp(-(rc / pr.sigma) ** 2)
    dG = G / pr.sigma if kernel == 0 else 2 * rc / pr.sigma ** 2 * G
    pn = np.sqrt(np.sum(p * p, axis=0))
    bv, bf = G * pn.sum(), dG * pn * pn.sum()
    eps, agree = (1e-12, 1e-12) if dtype == lm.F64 else (1e-5, TOL[lm.F32])
    slack = eps * max(np.max(np.abs(dq_o)), np.max(np.abs(dp_o)))
    dqs, dps = out[1]
    assert np.all(np.sqrt(np.sum((dqs - dq_o) ** 2, axis=0)) <= bv + slack)
    assert np.all(np.sqrt(np.sum((dps - dp_o) ** 2, axis=0)) <= bf + slack)
    print("sym against one-sided: %.2e %.2e" % (rel_err(dqs, out[0][0]), rel_err(dps, out[0][1])))
    assert rel_err(dqs, out[0][0]) <= agree and rel_err(dps, out[0][1]) <= agree
    assert np.max(np.abs(dqs - dq_o)) > 0.0      # something was skipped


@pytest.mark.parametrize("kernel,dtype", [(lm.CONON, lm.F64), (lm.GAUSS, lm.F64), (lm.CONON, lm.F32)])
def test_sym_cutoff_full_size_sampled_rows(kernel, dtype):
    """N = 65536 with tile skipping in the default launch shape (two row tiles, two waves,
    4-tile superblocks) at the radius where the kernel falls to 1e-16 (single precision:
    1e-10), Morton-ordered as lm_shoot orders it: sampled rows (both ends of a tile and the
    last point included) against the oracle, which computes rows one by one over all pairs."""
    n = 65536
    pr = inputs.config_sphere3d(n, kernel=kernel, sigma=0.05)
    perm = _morton_sorted(pr.X)
    q, p = rounded(pr.X[:, perm], dtype), rounded(pr.p_bench()[:, perm], dtype)
    L = np.log(1e16 if dtype == lm.F64 else 1e10)
    rc = pr.sigma * (L if kernel == 0 else np.sqrt(L))
    prm = lm.make_params(3, kernel, pr.sigma, cutoff=rc, dtype=dtype)
    plan = lm.lm_pair_plan(prm, n)
    assert plan["symmetric"] == 1 and plan["rows"] == 2 and plan["waves"] == 2
    qd, pd = dev(q, dtype), dev(p, dtype)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    lm.lm_rhs(prm, qd, pd, dq, dp)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(77).choice(n, 192, replace=False))
    idx = np.concatenate([[0, 63, 64, n - 1], idx])
    rq, rp = oracle.rhs_rows(q, p, idx, kernel, pr.sigma)
    eq = np.max(np.abs(host(dq)[:, idx] - rq)) / np.max(np.abs(rq))
    ep = np.max(np.abs(host(dp)[:, idx] - rp)) / np.max(np.abs(rp))
    print("cutoff full-size sampled kernel=%d dtype=%d: %.2e %.2e" % (kernel, dtype, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_sym_cutoff_shoot_matches_oracle(dtype):
    pr = inputs.config_sphere3d(3000, kernel=lm.GAUSS, sigma=0.1)
    q0, p0 = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    oq, op = oracle.shoot(q0, p0, lm.GAUSS, pr.sigma, 8)
    prm = lm.make_params(3, lm.GAUSS, pr.sigma, cutoff=pr.sigma * 36.9 ** 0.5, dtype=dtype)
    with _env(LM_SYM=1, LM_SYM_WAVES=2):
        q, p = dev(q0, dtype), dev(p0, dtype)
        q1, p1 = torch.empty_like(q), torch.empty_like(p)
        lm.lm_shoot(prm, q, p, 1.0, 8, q1, p1)
        torch.cuda.synchronize()
    assert rel_err(host(q1), oq) <= TOL[dtype] and rel_err(host(p1), op) <= TOL[dtype]
