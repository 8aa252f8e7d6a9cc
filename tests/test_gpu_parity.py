"""Parity of the HIP library with the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances (normwise per output array, max|gpu - oracle| / max|oracle|): 1e-10 for the
double-precision path and 1e-4 for the single-precision form, the bars the performance
target states.  Single-precision runs feed the oracle the same float-rounded inputs.
"""

import math

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1510_03816_amd as lm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {lm.F64: 1e-10, lm.F32: 1e-4}
TDT = {lm.F64: torch.float64, lm.F32: torch.float32}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def dev(a, dtype=lm.F64):
    return torch.tensor(np.ascontiguousarray(a), dtype=TDT[dtype], device=DEV)


def host(t):
    return t.detach().double().cpu().numpy()


def rounded(a, dtype):
    return a.astype(np.float32).astype(np.float64) if dtype == lm.F32 else a


def rel_err(got, want):
    scale = np.max(np.abs(want))
    d = np.max(np.abs(got - want))
    return d / scale if scale > 0 else d


def gpu_rhs(q, p, kernel, sigma, tau, dtype):
    prm = lm.make_params(q.shape[0], kernel, sigma, dtype=dtype, tau=tau)
    qd, pd = dev(q, dtype), dev(p, dtype)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    lm.lm_rhs(prm, qd, pd, dq, dp)
    torch.cuda.synchronize()
    return host(dq), host(dp)


# ------------------------------------------------------------------ right-hand side


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 1000, 4096])
def test_rhs_matches_oracle(n, dim, kernel, dtype):
    q, p = inputs.random_state(n, dim, seed=[100, n, dim], box=1.0, pscale=0.3)
    q, p = rounded(q, dtype), rounded(p, dtype)
    sigma, tau = (0.3 if dim == 3 else 0.25), 0.1
    dq_o, dp_o = oracle.rhs(q, p, kernel, sigma, tau)
    dq, dp = gpu_rhs(q, p, kernel, sigma, tau, dtype)
    print("n=%d dim=%d kernel=%d dtype=%d: %.2e %.2e" % (n, dim, kernel, dtype, rel_err(dq, dq_o), rel_err(dp, dp_o)))
    assert rel_err(dq, dq_o) <= TOL[dtype]
    assert rel_err(dp, dp_o) <= TOL[dtype]
    if n == 1:
        assert np.all(dp == 0.0)


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_rhs_coincident_particles(kernel):
    q, p = inputs.random_state(40, 2, seed=101)
    q[:, 10:20] = q[:, 0:10]          # ten pairs of coincident distinct particles
    dq_o, dp_o = oracle.rhs(q, p, kernel, 0.4)
    dq, dp = gpu_rhs(q, p, kernel, 0.4, 0.0, lm.F64)
    assert np.all(np.isfinite(dp))
    assert rel_err(dq, dq_o) <= 1e-10 and rel_err(dp, dp_o) <= 1e-10


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_rhs_full_size_sampled(kernel, dtype):
    """N = 65536 on the unit sphere (the 3-D workload) in the benchmark's launch shape;
    256 sampled rows are checked against the oracle, which computes rows one by one."""
    pr = inputs.config_sphere3d(65536, kernel=kernel)
    q, p = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    dq, dp = gpu_rhs(q, p, kernel, pr.sigma, 0.0, dtype)
    idx = np.sort(np.random.default_rng(102).choice(pr.n, 256, replace=False))
    idx = np.concatenate([[0, 63, 64, pr.n - 1], idx])
    rq, rp = oracle.rhs_rows(q, p, idx, kernel, pr.sigma)
    eq = np.max(np.abs(dq[:, idx] - rq)) / np.max(np.abs(rq))
    ep = np.max(np.abs(dp[:, idx] - rp)) / np.max(np.abs(rp))
    print("full-size sampled kernel=%d dtype=%d: %.2e %.2e" % (kernel, dtype, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]
    # the forces of the whole system sum to zero (antisymmetry), at any size
    if dtype == lm.F64:
        assert np.max(np.abs(dp.sum(axis=1))) <= 1e-9 * np.max(np.abs(dp))


# ------------------------------------------------------------------ shooting


SHOOT_CASES = [
    ("circle_ellipse_64", lambda: inputs.config_circle_ellipse(64), 100),
    ("curve2d_700", lambda: inputs.config_curve2d(700), 40),
    ("sphere3d_600_conon", lambda: inputs.config_sphere3d(600, sigma=0.2), 20),
    ("sphere3d_600_gauss", lambda: inputs.config_sphere3d(600, kernel=1, sigma=0.2), 20),
]


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("name,make,steps", SHOOT_CASES, ids=[c[0] for c in SHOOT_CASES])
def test_shoot_matches_oracle(name, make, steps, dtype):
    pr = make()
    q0, p0 = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    oq, op = oracle.shoot(q0, p0, pr.kernel, pr.sigma, steps)
    prm = lm.make_params(pr.dim, pr.kernel, pr.sigma, dtype=dtype)
    q, p = dev(q0, dtype), dev(p0, dtype)
    q1, p1 = torch.empty_like(q), torch.empty_like(p)
    lm.lm_shoot(prm, q, p, 1.0, steps, q1, p1)
    torch.cuda.synchronize()
    eq, ep = rel_err(host(q1), oq), rel_err(host(p1), op)
    print("%s dtype=%d: %.2e %.2e" % (name, dtype, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("n", [2, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257])
def test_small_problem_shoot_matches_oracle(n, dtype):
    """Small problems (up to 128 points) are shot in one launch (one workgroup, every stage in
    the kernel); sizes across its tile/chunk splits and the boundary to the stage-per-launch
    path, with the inexact term, against the oracle."""
    dim, kernel = (3, lm.GAUSS) if n % 2 else (2, lm.CONON)
    q0, p0 = inputs.random_state(n, dim, [310, n], box=1.0, pscale=0.3)
    q0, p0 = rounded(q0, dtype), rounded(p0, dtype)
    oq, op = oracle.shoot(q0, p0, kernel, 0.4, 25, T=0.9, tau=0.1)
    prm = lm.make_params(dim, kernel, 0.4, dtype=dtype, tau=0.1)
    q1, p1 = torch.empty_like(dev(q0, dtype)), torch.empty_like(dev(q0, dtype))
    lm.lm_shoot(prm, dev(q0, dtype), dev(p0, dtype), 0.9, 25, q1, p1)
    torch.cuda.synchronize()
    eq, ep = rel_err(host(q1), oq), rel_err(host(p1), op)
    print("n=%d dtype=%d: %.2e %.2e" % (n, dtype, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]


@pytest.mark.parametrize("waves", [4, 8, 16])
@pytest.mark.parametrize("n,dim,dtype", [(3, 2, lm.F64), (64, 3, lm.F64), (100, 2, lm.F64), (192, 2, lm.F64),
                                         (224, 3, lm.F64), (33, 2, lm.F32), (256, 3, lm.F32)])
def test_small_problem_shoot_every_width(n, dim, dtype, waves, monkeypatch):
    """The one-workgroup shoot at each of its widths (4, 8, 16 waves: one to four target tiles,
    1 to 16 source chunks; LM_SMALL = 1 takes it up to 256 points) against the oracle, on the
    structured workloads."""
    monkeypatch.setenv("LM_SMALL", "1")
    monkeypatch.setenv("LM_SMALL_WAVES", str(waves))
    pr = inputs.config_curve2d(n, sigma=0.3) if dim == 2 else inputs.config_sphere3d(n, kernel=lm.GAUSS, sigma=0.3)
    q0, p0 = rounded(pr.X, dtype), rounded(pr.p_bench(), dtype)
    oq, op = oracle.shoot(q0, p0, pr.kernel, pr.sigma, 40, tau=0.05)
    prm = lm.make_params(dim, pr.kernel, pr.sigma, dtype=dtype, tau=0.05)
    assert lm.lm_pair_plan(prm, n)["small"] == 1
    q1, p1 = torch.empty_like(dev(q0, dtype)), torch.empty_like(dev(q0, dtype))
    lm.lm_shoot(prm, dev(q0, dtype), dev(p0, dtype), 1.0, 40, q1, p1)
    torch.cuda.synchronize()
    eq, ep = rel_err(host(q1), oq), rel_err(host(p1), op)
    print("n=%d dim=%d dtype=%d waves=%d: %.2e %.2e" % (n, dim, dtype, waves, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]


def test_shoot_in_place_and_time_span():
    pr = inputs.config_curve2d(300)
    p0 = pr.p_bench()
    oq, op = oracle.shoot(pr.X, p0, 0, pr.sigma, 30, T=0.7, tau=0.2)
    prm = lm.make_params(2, lm.CONON, pr.sigma, tau=0.2)
    q, p = dev(pr.X), dev(p0)
    lm.lm_shoot(prm, q, p, 0.7, 30, q, p)           # outputs alias the inputs
    torch.cuda.synchronize()
    assert rel_err(host(q), oq) <= 1e-10 and rel_err(host(p), op) <= 1e-10


def test_single_particle_straight_line():
    prm = lm.make_params(3, lm.CONON, 0.1, tau=0.5)
    q = dev(np.array([[0.3], [-1.2], [2.0]]))
    p = dev(np.array([[0.7], [0.1], [-0.4]]))
    q1, p1 = torch.empty_like(q), torch.empty_like(p)
    lm.lm_shoot(prm, q, p, 1.0, 7, q1, p1)
    torch.cuda.synchronize()
    assert np.allclose(host(q1), host(q) + 1.5 * host(p), rtol=0, atol=1e-14)
    assert np.array_equal(host(p1), host(p))


def test_time_rescaling_predicts_longer_shoots():
    """The prediction property (momenta scaled by c reach, at t = 1, the state the unscaled
    momenta reach at t = c, with momenta scaled by c): shoot(X, c p0, T=1) equals
    (q, c p) of shoot(X, p0, T=c) with the same step count, on the GPU."""
    pr = inputs.config_curve2d(500)
    X, p0 = pr.X, pr.p_bench()
    prm = lm.make_params(2, lm.CONON, pr.sigma)
    c = 1.7
    a = [torch.empty_like(dev(X)) for _ in range(4)]
    lm.lm_shoot(prm, dev(X), dev(c * p0), 1.0, 60, a[0], a[1])
    lm.lm_shoot(prm, dev(X), dev(p0), c, 60, a[2], a[3])
    torch.cuda.synchronize()
    assert rel_err(host(a[0]), host(a[2])) <= 1e-12
    assert rel_err(host(a[1]), c * host(a[3])) <= 1e-12


def test_shoot_is_deterministic():
    pr = inputs.config_curve2d(2000)
    prm = lm.make_params(2, lm.CONON, pr.sigma)
    q, p = dev(pr.X), dev(pr.p_bench())
    outs = []
    for _ in range(2):
        q1, p1 = torch.empty_like(q), torch.empty_like(p)
        lm.lm_shoot(prm, q, p, 1.0, 10, q1, p1)
        torch.cuda.synchronize()
        outs.append((host(q1), host(p1)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_full_size_shoot_conserves_momentum_and_energy(kernel):
    """At N = 65536 the oracle cannot shoot in seconds; properties that hold at any size
    are checked instead: total momentum is exact, H drifts at RK4 order."""
    pr = inputs.config_sphere3d(65536, kernel=kernel)
    prm = lm.make_params(3, kernel, pr.sigma)
    q, p = dev(pr.X), dev(pr.p_bench())
    H0 = lm.lm_hamiltonian(prm, q, p)
    q1, p1 = torch.empty_like(q), torch.empty_like(p)
    lm.lm_shoot(prm, q, p, 1.0, 4, q1, p1)
    H1 = lm.lm_hamiltonian(prm, q1, p1)
    P0, P1 = host(p).sum(axis=1), host(p1).sum(axis=1)
    print("kernel %d: H %.10e -> %.10e, sum p drift %.2e" % (kernel, H0, H1, np.max(np.abs(P1 - P0))))
    assert np.max(np.abs(P1 - P0)) <= 1e-11 * np.max(np.abs(host(p))) * pr.n
    assert abs(H1 - H0) <= 1e-6 * abs(H0)


# ------------------------------------------------------------------ Hamiltonian, velocity, K-solve


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("dim,kernel", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_hamiltonian_matches_oracle(dim, kernel, dtype):
    q, p = inputs.random_state(777, dim, seed=[103, dim], pscale=0.2)
    q, p = rounded(q, dtype), rounded(p, dtype)
    prm = lm.make_params(dim, kernel, 0.3, dtype=dtype)
    H = lm.lm_hamiltonian(prm, dev(q, dtype), dev(p, dtype))
    assert H == pytest.approx(oracle.hamiltonian(q, p, kernel, 0.3), rel=1e-10)


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("dim,kernel", [(2, 0), (3, 1)])
def test_velocity_field_matches_oracle(dim, kernel, dtype):
    q, p = inputs.random_state(500, dim, seed=[104, dim])
    x, _ = inputs.random_state(333, dim, seed=[105, dim], box=1.5)
    q, p, x = rounded(q, dtype), rounded(p, dtype), rounded(x, dtype)
    prm = lm.make_params(dim, kernel, 0.3, dtype=dtype)
    u = torch.empty((dim, 333), dtype=TDT[dtype], device=DEV)
    lm.lm_velocity(prm, dev(q, dtype), dev(p, dtype), dev(x, dtype), u)
    torch.cuda.synchronize()
    assert rel_err(host(u), oracle.velocity(q, p, x, kernel, 0.3)) <= TOL[dtype]


@pytest.mark.parametrize("name,make", [
    ("circle_ellipse_64", lambda: inputs.config_circle_ellipse(64)),
    ("curve2d_1000", lambda: inputs.config_curve2d(1000)),
    ("example1_64", lambda: inputs.Problem("ex1", inputs.example1(64)[0], None, 0, 1.0, 50)),
])
def test_ksolve_matches_cholesky(name, make):
    pr = make()
    X = pr.X
    b = np.random.default_rng(106).standard_normal(X.shape)
    st, L = oracle.cholesky(oracle.kmatrix(X, pr.kernel, pr.sigma))
    assert st == 0
    want = np.stack([oracle.cholesky_solve(L, b[c]) for c in range(X.shape[0])])
    prm = lm.make_params(X.shape[0], pr.kernel, pr.sigma)
    x = torch.empty((X.shape[0], X.shape[1]), dtype=torch.float64, device=DEV)
    it = lm.lm_ksolve(prm, dev(X), dev(b), x, rtol=1e-13, solver=lm.SOLVE_CG)
    print("%s: %d CG iterations, rel err %.2e" % (name, it, rel_err(host(x), want)))
    assert rel_err(host(x), want) <= 1e-8
    xd = torch.empty_like(x)
    assert lm.lm_ksolve(prm, dev(X), dev(b), xd, solver=lm.SOLVE_DENSE) == 0
    print("%s: dense rel err %.2e" % (name, rel_err(host(xd), want)))
    assert rel_err(host(xd), want) <= 1e-9


# ------------------------------------------------------------------ feedback matching


def gpu_match(X, Y, kernel, sigma, h, tol, steps, dtype=lm.F64, max_iter=500, tau=0.0, stop_rule=0):
    prm = lm.make_params(X.shape[0], kernel, sigma, dtype=dtype, tau=tau)
    p0 = torch.zeros(X.shape, dtype=torch.float64, device=DEV)
    st, info, hist = lm.lm_feedback_match(prm, dev(X), dev(Y), p0, h=h, tol=tol, steps=steps,
                                          max_iter=max_iter, stop_rule=stop_rule)
    return st, info, hist, host(p0)


def test_feedback_circle_to_ellipse_matches_oracle():
    pr = inputs.config_circle_ellipse(64)
    st, info, hist, p0 = gpu_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-6, pr.steps)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-6, pr.steps)
    print("gpu %d its (%d CG) resid %.3e H %.8f | oracle %d its resid %.3e H %.8f" % (
        info.iters, info.cg_iters, info.resid_inf, info.H, ref.iters, ref.resid, ref.H))
    assert st == 0 and ref.status == 0
    assert info.iters == ref.iters
    assert rel_err(p0, ref.p0) <= 1e-8
    assert info.H == pytest.approx(ref.H, rel=1e-9)
    assert np.allclose(hist, ref.hist, rtol=1e-6, atol=1e-12)


def test_feedback_example1_reproduces_paper_count():
    X, Y = inputs.example1(64)
    st, info, _, p0 = gpu_match(X, Y, 0, 1.0, 0.3, 1e-3, 50)
    assert st == 0 and info.iters == 197
    assert float("%.1e" % info.resid_inf) == 9.5e-4
    assert 2 * info.H == pytest.approx(46.5022, rel=1e-4)


def test_feedback_table2_divergence_is_reported():
    X, Y = inputs.example2(64)
    st, info, hist, _ = gpu_match(X, Y, 0, 1.0, 1.1, 1e-3, 50)
    assert st == lm.LM_EDIVERGED
    st, info, hist, _ = gpu_match(X, Y, 0, 1.0, 0.8, 1e-3, 50)
    assert st == 0 and info.iters == 18


def test_feedback_single_precision_shoot():
    pr = inputs.config_circle_ellipse(64)
    st, info, _, p0 = gpu_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-5, pr.steps, dtype=lm.F32)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-5, pr.steps)
    assert st == 0 and abs(info.iters - ref.iters) <= 1
    assert rel_err(p0, ref.p0) <= 1e-4


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_match_from_rest_does_not_integrate_the_first_shoot(dtype):
    """Zero initial momenta (Algorithm 1's start) leave every landmark at rest, every term of
    the right-hand side having a momentum factor, so the first shoot is the identity map: the
    match integrates one shoot fewer than its updates + 1, its first residual is max|Y - X|
    exactly, and its iteration count and momenta are the oracle's, which integrates that
    shoot (FP32, on the well-conditioned circle -> ellipse as the single-precision test above:
    the oracle's count or one more, momenta to 1e-4).  From non-zero momenta every shoot is
    integrated."""
    if dtype == lm.F64:
        pr, tol, steps = inputs.config_curve2d(700), 1e-6, 40
    else:
        pr, tol = inputs.config_circle_ellipse(64), 1e-5
        steps = pr.steps
    prm = lm.make_params(2, lm.CONON, pr.sigma, dtype=dtype)
    p0 = torch.zeros((2, pr.n), dtype=torch.float64, device=DEV)
    st, info, hist = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=tol, steps=steps,
                                          max_iter=200)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, tol, steps, max_iter=200)
    assert st == 0 and ref.status == 0
    assert info.shoots == info.iters
    assert hist[0] == np.max(np.abs(pr.Y - pr.X))
    if dtype == lm.F64:
        assert info.iters == ref.iters
        assert rel_err(host(p0), ref.p0) <= 1e-8
    else:
        assert 0 <= info.iters - ref.iters <= 1
        assert rel_err(host(p0), ref.p0) <= 1e-4
    p_start = dev(0.5 * ref.p0)
    st2, info2, hist2 = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p_start, h=0.8, tol=tol, steps=steps,
                                             max_iter=200)
    assert st2 == 0
    assert info2.shoots == info2.iters + 1 == len(hist2)


def test_feedback_single_precision_switches_to_double():
    """With f32_switch the match shoots in single precision until the residual is below the
    switch, then in double: it reaches a tolerance single precision cannot, in the oracle's
    iteration count (or one more), and its last shoot is a double-precision one."""
    pr = inputs.config_curve2d(700)
    prm = lm.make_params(2, lm.CONON, pr.sigma, dtype=lm.F32)
    p0 = torch.zeros((2, pr.n), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, info, shots = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=1e-9, steps=40, max_iter=200,
                                           q1=q1, f32_switch=1e-4)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-9, 40, max_iter=200)
    print("switch: gpu %d updates, %d shoots, resid %.2e | oracle %d" % (info.iters, len(shots), info.resid_inf,
                                                                           ref.iters))
    assert st == 0 and ref.status == 0
    assert 0 <= info.iters - ref.iters <= 1
    assert info.iters + 1 <= len(shots) <= info.iters + 2
    assert info.resid_inf < 1e-9
    oq, _ = oracle.shoot(pr.X, host(p0), 0, pr.sigma, 40)
    assert rel_err(host(q1), oq) <= 1e-10


def test_feedback_single_precision_floor_switches_to_double():
    """A switch threshold below what single-precision shoots resolve (1e-12, against a floor of
    about 1e-5 on this curve): the residual stops falling at the floor, the match re-shoots in
    double precision there and reaches tol = 1e-9 within two updates of the oracle's count
    (either way: the single-precision updates before the switch move its residuals slightly)."""
    pr = inputs.config_curve2d(700)
    prm = lm.make_params(2, lm.CONON, pr.sigma, dtype=lm.F32)
    p0 = torch.zeros((2, pr.n), dtype=torch.float64, device=DEV)
    st, info, hist = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=1e-9, steps=40, max_iter=200,
                                          f32_switch=1e-12)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-9, 40, max_iter=200)
    print("floor switch: gpu %d updates, %d shoots | oracle %d; residuals %s" % (
        info.iters, info.shoots, ref.iters, " ".join("%.1e" % h for h in hist)))
    assert st == 0 and ref.status == 0
    assert info.resid_inf < 1e-9
    assert abs(info.iters - ref.iters) <= 2


@pytest.mark.parametrize("tau,solver", [(0.05, lm.SOLVE_DENSE), (0.3, lm.SOLVE_DENSE), (0.3, lm.SOLVE_CG)])
def test_feedback_inexact_matches_oracle(tau, solver):
    """Inexact matching (eq. N-particle-inexact, Table 5's stopping rule on successive
    momenta): the same iteration count, momenta and residual history as the oracle."""
    X, Y = inputs.example2(64)
    prm = lm.make_params(2, lm.CONON, 1.0, tau=tau)
    p0 = torch.zeros((2, 64), dtype=torch.float64, device=DEV)
    st, info, hist = lm.lm_feedback_match(prm, dev(X), dev(Y), p0, h=0.8, tol=1e-3, steps=30, max_iter=300,
                                          stop_rule=1, solver=solver)
    ref = oracle.feedback_match(X, Y, 0, 1.0, 0.8, 1e-3, 30, max_iter=300, tau=tau, stop_rule=1)
    print("inexact tau=%g: gpu %d its resid %.3e | oracle %d its resid %.3e" % (tau, info.iters, info.resid_inf,
                                                                              ref.iters, ref.resid))
    assert st == 0 and ref.status == 0
    assert info.iters == ref.iters
    assert rel_err(host(p0), ref.p0) <= 1e-8
    assert np.allclose(hist, ref.hist, rtol=1e-6, atol=1e-12)


def test_feedback_max_iter_reports_not_converged():
    pr = inputs.config_circle_ellipse(64)
    st, info, _, _ = gpu_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-6, pr.steps, max_iter=3)
    assert st == lm.LM_ENOTCONV and info.iters == 3


def test_bad_arguments_raise():
    prm = lm.make_params(2, lm.CONON, 0.5)
    q = torch.zeros((2, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        lm.lm_rhs(prm, q, q[:, :5].contiguous(), torch.empty_like(q), torch.empty_like(q))
    with pytest.raises(lm.LmError):
        lm.lm_shoot(prm, q, q.clone(), 1.0, 0, torch.empty_like(q), torch.empty_like(q))


def test_feedback_step_matches_oracle_iterates():
    """Three calls of the one-iteration entry point equal three updates of Algorithm 1."""
    pr = inputs.config_circle_ellipse(64)
    prm = lm.make_params(2, lm.CONON, pr.sigma)
    X, Y = dev(pr.X), dev(pr.Y)
    p = torch.zeros_like(X)
    resids = []
    for _ in range(3):
        st, info = lm.lm_feedback_step(prm, X, Y, p, h=0.8, tol=1e-6, steps=pr.steps)
        assert st == 0 and info.converged == 0 and info.cg_iters > 0 and info.shoot_ms > 0
        resids.append(info.resid_inf)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-6, pr.steps, max_iter=3)
    assert ref.status == oracle.ENOTCONV and ref.iters == 3
    assert np.allclose(resids, ref.hist[:3], rtol=1e-8, atol=0)
    assert rel_err(host(p), ref.p0) <= 1e-9


# ------------------------------------------------------------------ cutoff mode (tile skipping)


def _morton_sorted(X):
    """Reorder a point set spatially (Morton order) so that 64-point tiles are compact."""
    lo, hi = X.min(axis=1, keepdims=True), X.max(axis=1, keepdims=True)
    g = np.clip(((X - lo) / (hi - lo) * 1023).astype(np.int64), 0, 1023)
    key = np.zeros(X.shape[1], dtype=np.int64)
    for b in range(10):
        for c in range(X.shape[0]):
            key |= ((g[c] >> b) & 1) << (X.shape[0] * b + c)
    return np.argsort(key, kind="stable")


def _cutoff_bound(kernel, sigma, rc, p):
    """Certified bounds on what skipping pairs farther apart than rc can drop, per target:
    velocity <= G(rc) sum_j |p_j|, force <= |G'(rc)| |p_i| sum_j |p_j| (G and |G'| decrease
    beyond rc; for the Gaussian that needs rc >= sigma/sqrt 2)."""
    G = math.exp(-rc / sigma) if kernel == 0 else math.exp(-(rc / sigma) ** 2)
    dG = G / sigma if kernel == 0 else 2 * rc / sigma ** 2 * G
    pn = np.sqrt(np.sum(p * p, axis=0))
    return G * pn.sum(), dG * pn * pn.sum()


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_rhs_cutoff_at_negligible_radius_meets_exact_parity(kernel, dtype):
    """Skipping tiles beyond a radius where the kernel is below 1e-16 keeps the exact bar."""
    pr = inputs.config_sphere3d(20000, kernel=kernel, sigma=0.05)
    perm = _morton_sorted(pr.X)
    q, p = rounded(pr.X[:, perm], dtype), rounded(pr.p_bench()[:, perm], dtype)
    rc = pr.sigma * (36.9 if kernel == 0 else math.sqrt(36.9))
    dq_o, dp_o = oracle.rhs(q, p, kernel, pr.sigma)
    prm = lm.make_params(3, kernel, pr.sigma, dtype=dtype, cutoff=rc)
    qd, pd = dev(q, dtype), dev(p, dtype)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    lm.lm_rhs(prm, qd, pd, dq, dp)
    torch.cuda.synchronize()
    eq, ep = rel_err(host(dq), dq_o), rel_err(host(dp), dp_o)
    print("cutoff rc=%.3f kernel=%d dtype=%d: %.2e %.2e" % (rc, kernel, dtype, eq, ep))
    assert eq <= TOL[dtype] and ep <= TOL[dtype]


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_rhs_cutoff_error_within_certified_bound(kernel):
    pr = inputs.config_sphere3d(8000, kernel=kernel, sigma=0.05)
    perm = _morton_sorted(pr.X)
    q, p = pr.X[:, perm], pr.p_bench()[:, perm]
    rc = 3.0 * pr.sigma
    dq_o, dp_o = oracle.rhs(q, p, kernel, pr.sigma)
    prm = lm.make_params(3, kernel, pr.sigma, cutoff=rc)
    qd, pd = dev(q), dev(p)
    dq, dp = torch.empty_like(qd), torch.empty_like(pd)
    lm.lm_rhs(prm, qd, pd, dq, dp)
    torch.cuda.synchronize()
    bv, bf = _cutoff_bound(kernel, pr.sigma, rc, p)
    errv = np.sqrt(np.sum((host(dq) - dq_o) ** 2, axis=0))
    errf = np.sqrt(np.sum((host(dp) - dp_o) ** 2, axis=0))
    slack = 1e-12 * max(np.max(np.abs(dq_o)), np.max(np.abs(dp_o)))
    print("kernel %d: max err v %.2e (bound %.2e), f %.2e (bound max %.2e)" % (
        kernel, errv.max(), bv, errf.max(), bf.max()))
    assert np.all(errv <= bv + slack)
    assert np.all(errf <= bf + slack)
    assert errv.max() > 0.0        # something was skipped at this radius


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_shoot_cutoff_reorders_internally_and_matches(kernel):
    """lm_shoot sorts the points itself in cutoff mode: unsorted input, outputs in the input
    order, exact parity at a negligible radius."""
    pr = inputs.config_sphere3d(3000, kernel=kernel, sigma=0.1)
    q0, p0 = pr.X, pr.p_bench()
    oq, op = oracle.shoot(q0, p0, kernel, pr.sigma, 8)
    rc = pr.sigma * (36.9 if kernel == 0 else math.sqrt(36.9))
    prm = lm.make_params(3, kernel, pr.sigma, cutoff=rc)
    q, p = dev(q0), dev(p0)
    q1, p1 = torch.empty_like(q), torch.empty_like(p)
    lm.lm_shoot(prm, q, p, 1.0, 8, q1, p1)
    torch.cuda.synchronize()
    assert rel_err(host(q1), oq) <= 1e-10 and rel_err(host(p1), op) <= 1e-10


def test_velocity_cutoff_matches():
    q, p = inputs.random_state(3000, 2, seed=107, box=2.0)
    x, _ = inputs.random_state(1000, 2, seed=108, box=2.0)
    pq, px = _morton_sorted(q), _morton_sorted(x)
    q, p, x = q[:, pq], p[:, pq], x[:, px]
    rc = 0.05 * 36.9
    prm = lm.make_params(2, lm.CONON, 0.05, cutoff=rc)
    u = torch.empty((2, 1000), dtype=torch.float64, device=DEV)
    lm.lm_velocity(prm, dev(q), dev(p), dev(x), u)
    torch.cuda.synchronize()
    assert rel_err(host(u), oracle.velocity(q, p, x, 0, 0.05)) <= 1e-10


def test_feedback_cutoff_matches_exact_iteration():
    pr = inputs.config_curve2d(1500)
    rc = pr.sigma * 36.9
    prm = lm.make_params(2, lm.CONON, pr.sigma, cutoff=rc)
    p0 = torch.zeros((2, pr.n), dtype=torch.float64, device=DEV)
    st, info, hist = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=1e-6, steps=20, max_iter=60)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-6, 20, max_iter=60)
    assert st == 0 and ref.status == 0 and info.iters == ref.iters
    assert rel_err(host(p0), ref.p0) <= 1e-8


@pytest.mark.parametrize("sweeps", ["block", "super"])
@pytest.mark.parametrize("n,dim,kernel,sigma,tau", [
    (1, 2, 0, 0.5, 0.0), (127, 2, 0, 0.5, 0.0), (128, 3, 1, 0.4, 0.0), (129, 2, 0, 0.2, 0.3),
    (333, 3, 0, 0.3, 0.0), (1000, 2, 0, 0.1, 0.0), (1024, 3, 0, 0.15, 0.0), (1100, 3, 1, 0.1, 0.05),
    (2500, 3, 0, 0.15, 0.1), (3072, 2, 0, 0.1, 0.0),
])
def test_dense_ksolve_matches_cholesky(n, dim, kernel, sigma, tau, sweeps, monkeypatch):
    """Blocked GPU Cholesky (MFMA trailing updates) against the oracle's textbook Cholesky,
    across panel boundaries and ragged tails, with both solve forms: one launch per 128-row
    block, and superblocks of 8 blocks through their stored inverses (forced on at every size
    here: one superblock up to 1024 points, a ragged second from 1025)."""
    monkeypatch.setenv("LM_DENSE_SUPER", "1" if sweeps == "super" else "0")
    X = inputs.fibonacci_sphere(n) if dim == 3 else inputs.config_curve2d(n).X
    b = np.random.default_rng([109, n]).standard_normal(X.shape)
    K = oracle.kmatrix(X, kernel, sigma) + tau * np.eye(n)
    st, L = oracle.cholesky(K)
    assert st == 0
    want = np.stack([oracle.cholesky_solve(L, b[c]) for c in range(dim)])
    prm = lm.make_params(dim, kernel, sigma, tau=tau)
    x = dev(b)
    lm.lm_ksolve(prm, dev(X), x, x, solver=lm.SOLVE_DENSE)       # in place
    ev = np.linalg.eigvalsh(K)          # K is symmetric positive definite
    cond = ev[-1] / ev[0]
    err = rel_err(host(x), want)
    print("n=%d cond %.1e dense rel err %.2e" % (n, cond, err))
    assert err <= max(1e-12, 1e-15 * cond)


@pytest.mark.parametrize("sweeps", ["block", "super"])
def test_dense_ksolve_several_trailing_updates_matches_cg(sweeps, monkeypatch):
    """N = 5000: three trailing updates on 128 x 128 tiles (the last tile row ragged), checked
    against conjugate gradients on the same system (matrix-free, through the pair kernel);
    both solve forms (superblocks: five, the last ragged)."""
    monkeypatch.setenv("LM_DENSE_SUPER", "1" if sweeps == "super" else "0")
    n = 5000
    X = inputs.fibonacci_sphere(n)
    b = np.random.default_rng([113, n]).standard_normal(X.shape)
    prm = lm.make_params(3, lm.CONON, 0.15, tau=0.1)
    xd, xc = (torch.empty((3, n), dtype=torch.float64, device=DEV) for _ in range(2))
    assert lm.lm_ksolve(prm, dev(X), dev(b), xd, solver=lm.SOLVE_DENSE) == 0
    it = lm.lm_ksolve(prm, dev(X), dev(b), xc, solver=lm.SOLVE_CG, rtol=1e-13, max_iter=5000)
    err = rel_err(host(xd), host(xc))
    print("n=%d dense vs CG (%d iterations) rel diff %.2e" % (n, it, err))
    assert err <= 1e-9


@pytest.mark.parametrize("n,dim,sigma,tau", [(2500, 3, 0.15, 0.1), (5000, 3, 0.15, 0.1), (3000, 2, 0.1, 0.0)])
def test_dense_ksolve_with_single_precision_updates(n, dim, sigma, tau, monkeypatch):
    """The factor whose trailing updates multiply in single precision (matches with FP32 shoots
    use it; LM_FACTOR_F32 = 1 forces it here): one (n = 2500) to three (n = 5000) updates take
    that path, the rest and the diagonal blocks stay in double.  Against the oracle's Cholesky
    solve the relative error stays within cond(K) times 1e-6, the single-precision rounding of
    the updates carried through the solve."""
    monkeypatch.setenv("LM_FACTOR_F32", "1")
    X = inputs.fibonacci_sphere(n) if dim == 3 else inputs.config_curve2d(n).X
    b = np.random.default_rng([131, n]).standard_normal(X.shape)
    K = oracle.kmatrix(X, lm.CONON, sigma) + tau * np.eye(n)
    st, L = oracle.cholesky(K)
    assert st == 0
    want = np.stack([oracle.cholesky_solve(L, b[c]) for c in range(dim)])
    ev = np.linalg.eigvalsh(K)
    cond = ev[-1] / ev[0]
    prm = lm.make_params(dim, lm.CONON, sigma, tau=tau)
    x = dev(b)
    lm.lm_ksolve(prm, dev(X), x, x, solver=lm.SOLVE_DENSE)
    err = rel_err(host(x), want)
    print("n=%d cond %.1e single-precision updates: rel err %.2e" % (n, cond, err))
    assert err <= 1e-6 * cond
    monkeypatch.setenv("LM_FACTOR_F32", "0")
    x64 = dev(b)
    lm.lm_ksolve(prm, dev(X), x64, x64, solver=lm.SOLVE_DENSE)
    assert rel_err(host(x64), want) <= max(1e-12, 1e-15 * cond)


@pytest.mark.parametrize("n,dim", [(2500, 3), (5000, 3), (3001, 2)])
def test_single_precision_updates_from_the_float_panel_copy_are_bitwise_the_same(n, dim, monkeypatch):
    """The single-precision trailing updates stage a float copy of each update's operand
    columns (ragged tiles at the end, rows past n read as zero); staged from the FP64 matrix
    and rounded on the way into LDS (LM_FACTOR_F32_PANEL = 0) they multiply the same floats in
    the same order, so the solves agree bit for bit."""
    monkeypatch.setenv("LM_FACTOR_F32", "1")
    X = inputs.fibonacci_sphere(n) if dim == 3 else inputs.config_curve2d(n).X
    b = np.random.default_rng([132, n]).standard_normal(X.shape)
    prm = lm.make_params(dim, lm.CONON, 0.15, tau=0.1)
    out = []
    for panel in ("1", "0"):
        monkeypatch.setenv("LM_FACTOR_F32_PANEL", panel)
        x = dev(b)
        lm.lm_ksolve(prm, dev(X), x, x, solver=lm.SOLVE_DENSE)
        out.append(host(x))
    assert np.all(np.isfinite(out[0])) and np.array_equal(out[0], out[1])


def test_mixed_precision_match_with_single_precision_factor_updates():
    """A match with FP32 shoots switching to FP64 on a 2600-point curve, whose dense factor
    takes a single-precision trailing update: it reaches tol = 1e-8 with an FP64 residual in
    the oracle's iteration count or one more, and its q(1) is the oracle's shoot of the
    momenta it returns."""
    pr = inputs.config_curve2d(2600)
    prm = lm.make_params(2, lm.CONON, pr.sigma, dtype=lm.F32)
    p0 = torch.zeros((2, pr.n), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, info, hist = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=1e-8, steps=20, max_iter=200,
                                          q1=q1, f32_switch=1e-4)
    ref = oracle.feedback_match(pr.X, pr.Y, 0, pr.sigma, 0.8, 1e-8, 20, max_iter=200)
    print("mixed 2600: gpu %d updates | oracle %d" % (info.iters, ref.iters))
    assert st == 0 and ref.status == 0
    assert abs(info.iters - ref.iters) <= 1
    assert info.resid_inf < 1e-8
    oq, _ = oracle.shoot(pr.X, host(p0), 0, pr.sigma, 20)
    assert rel_err(host(q1), oq) <= 1e-10


def test_dense_ksolve_reports_singular_kernel_matrix():
    X = np.zeros((2, 300))          # every point at the origin: K is the all-ones matrix
    X[0, :] = np.linspace(0, 1e-9, 300)
    prm = lm.make_params(2, lm.GAUSS, 1.0)
    x = torch.empty((2, 300), dtype=torch.float64, device=DEV)
    with pytest.raises(lm.LmError) as e:
        lm.lm_ksolve(prm, dev(X), dev(np.ones((2, 300))), x, solver=lm.SOLVE_DENSE)
    assert e.value.status == lm.LM_ESINGULAR


def test_dense_ksolve_at_16384_matches_cg():
    """N = 16384 on the 3-D sphere workload (sigma 0.05): 128 panels, 16 trailing updates on
    128 x 128 tiles, the forward sweep on the transposed panel copies; against conjugate
    gradients on the same system."""
    pr = inputs.config_sphere3d(16384)
    prm = lm.make_params(3, lm.CONON, pr.sigma)
    b = np.random.default_rng([114, pr.n]).standard_normal(pr.X.shape)
    xd, xc = (torch.empty((3, pr.n), dtype=torch.float64, device=DEV) for _ in range(2))
    assert lm.lm_ksolve(prm, dev(pr.X), dev(b), xd, solver=lm.SOLVE_DENSE) == 0
    it = lm.lm_ksolve(prm, dev(pr.X), dev(b), xc, solver=lm.SOLVE_CG, rtol=1e-13, max_iter=5000)
    err = rel_err(host(xd), host(xc))
    print("n=%d dense vs CG (%d iterations) rel diff %.2e" % (pr.n, it, err))
    assert err <= 1e-9


def test_dense_ksolve_refuses_sizes_beyond_the_factor_limit():
    """n = 2^21 points: the trailing update addresses 128 rows of the factor with 31-bit byte
    offsets, so a forced dense solve is refused (LM_ENOMEM) before anything is allocated or
    launched; nothing is read from the inputs."""
    n = 1 << 21
    prm = lm.make_params(2, lm.CONON, 0.1)
    X = torch.zeros((2, n), dtype=torch.float64, device=DEV)
    x = torch.empty_like(X)
    with pytest.raises(lm.LmError) as e:
        lm.lm_ksolve(prm, X, X, x, solver=lm.SOLVE_DENSE)
    assert e.value.status == lm.LM_ENOMEM


def test_feedback_with_cg_solver_matches_dense():
    pr = inputs.config_circle_ellipse(64)
    prm = lm.make_params(2, lm.CONON, pr.sigma)
    out = {}
    for solver in (lm.SOLVE_CG, lm.SOLVE_DENSE):
        p0 = torch.zeros((2, 64), dtype=torch.float64, device=DEV)
        st, info, hist = lm.lm_feedback_match(prm, dev(pr.X), dev(pr.Y), p0, h=0.8, tol=1e-6, steps=pr.steps,
                                              solver=solver)
        assert st == 0
        out[solver] = (info.iters, host(p0))
    assert out[lm.SOLVE_CG][0] == out[lm.SOLVE_DENSE][0]
    assert rel_err(out[lm.SOLVE_CG][1], out[lm.SOLVE_DENSE][1]) <= 1e-9


# ------------------------------------------------------------------ reverse mode (adjoint)


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 17, 65, 1000])
def test_rhs_vjp_matches_oracle(n, dim, kernel):
    q, p = inputs.random_state(n, dim, seed=[110, n, dim], pscale=0.3)
    rng = np.random.default_rng([111, n])
    a, b = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
    prm = lm.make_params(dim, kernel, 0.3, tau=0.2)
    aq, ap = torch.empty((dim, n), dtype=torch.float64, device=DEV), torch.empty((dim, n), dtype=torch.float64, device=DEV)
    lm.lm_rhs_vjp(prm, dev(q), dev(p), dev(a), dev(b), aq, ap)
    torch.cuda.synchronize()
    oq, op = oracle.rhs_vjp(q, p, a, b, kernel, 0.3, 0.2)
    print("vjp n=%d dim=%d kernel=%d: %.2e %.2e" % (n, dim, kernel, rel_err(host(aq), oq), rel_err(host(ap), op)))
    assert rel_err(host(aq), oq) <= 1e-10 and rel_err(host(ap), op) <= 1e-10


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
@pytest.mark.parametrize("ckpt", [0, 1, 7, 20])
def test_shoot_adjoint_matches_oracle(kernel, ckpt):
    pr = inputs.config_sphere3d(300, kernel=kernel, sigma=0.3)
    q0, p0 = pr.X, pr.p_bench()
    rng = np.random.default_rng(112)
    gq1, gp1 = rng.standard_normal(q0.shape), rng.standard_normal(q0.shape)
    oq, op = oracle.shoot_adjoint(q0, p0, gq1, gp1, kernel, pr.sigma, 20, T=0.8, tau=0.1)
    prm = lm.make_params(3, kernel, pr.sigma, tau=0.1)
    gq0, gp0 = torch.empty((3, 300), dtype=torch.float64, device=DEV), torch.empty((3, 300), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(gq0)
    lm.lm_shoot_adjoint(prm, dev(q0), dev(p0), 0.8, 20, ckpt, dev(gq1), dev(gp1), gq0, gp0, q1=q1)
    torch.cuda.synchronize()
    fq, _ = oracle.shoot(q0, p0, kernel, pr.sigma, 20, T=0.8, tau=0.1)
    print("adjoint kernel=%d ckpt=%d: %.2e %.2e" % (kernel, ckpt, rel_err(host(gq0), oq), rel_err(host(gp0), op)))
    assert rel_err(host(gq0), oq) <= 1e-10 and rel_err(host(gp0), op) <= 1e-10
    assert rel_err(host(q1), fq) <= 1e-10


@pytest.mark.parametrize("kernel", [lm.CONON, lm.GAUSS])
def test_energy_gradient_matches_oracle(kernel):
    pr = inputs.config_sphere3d(500, kernel=kernel, sigma=0.2)
    p0 = 0.3 * pr.p_bench()
    E_o, g_o = oracle.energy_and_grad(pr.X, pr.Y, p0, kernel, pr.sigma, 100.0, 10)
    prm = lm.make_params(3, kernel, pr.sigma)
    g = torch.empty((3, 500), dtype=torch.float64, device=DEV)
    E = lm.lm_energy_grad(prm, dev(pr.X), dev(pr.Y), dev(p0), 100.0, 10, g, ckpt_every=3)
    assert E == pytest.approx(E_o, rel=1e-11)
    assert rel_err(host(g), g_o) <= 1e-10


def test_energy_gradient_at_rest_closed_form():
    """At p0 = 0 the flow is at rest and its linearisation is q(1) = X + K(X) dp exactly, so
    the gradient is lam K(X) (X - Y)."""
    pr = inputs.config_adjoint3d(1024)
    prm = lm.make_params(3, lm.GAUSS, pr.sigma)
    g = torch.empty((3, pr.n), dtype=torch.float64, device=DEV)
    E = lm.lm_energy_grad(prm, dev(pr.X), dev(pr.Y), dev(np.zeros_like(pr.X)), 100.0, 10, g, ckpt_every=10)
    K = oracle.kmatrix(pr.X, 1, pr.sigma)
    want = 100.0 * (K @ (pr.X - pr.Y).T).T
    assert rel_err(host(g), want) <= 1e-12
    assert E == pytest.approx(50.0 * np.sum((pr.X - pr.Y) ** 2), rel=1e-13)


def test_energy_gradient_finite_differences_on_subset():
    """Central differences of E on 32 seeded particle indices x 3 components (the
    differentiation workload's check, at reduced N)."""
    pr = inputs.config_adjoint3d(2048)
    prm = lm.make_params(3, lm.GAUSS, pr.sigma)
    X, Y = dev(pr.X), dev(pr.Y)
    p = 0.3 * pr.p_bench()
    g = torch.empty((3, pr.n), dtype=torch.float64, device=DEV)
    lm.lm_energy_grad(prm, X, Y, dev(p), 100.0, 20, g, ckpt_every=10)
    gh = host(g)
    scratch = torch.empty_like(g)
    eps = 1e-5
    worst = 0.0
    for i in pr.extra["fd_idx"]:
        for c in range(3):
            e = np.zeros_like(p)
            e[c, i] = eps
            Ep = lm.lm_energy_grad(prm, X, Y, dev(p + e), 100.0, 20, scratch, ckpt_every=10)
            Em = lm.lm_energy_grad(prm, X, Y, dev(p - e), 100.0, 20, scratch, ckpt_every=10)
            fd = (Ep - Em) / (2 * eps)
            worst = max(worst, abs(fd - gh[c, i]) / max(abs(gh[c, i]), 1e-3 * np.abs(gh).max()))
    print("FD worst relative difference %.2e" % worst)
    assert worst <= 1e-6


def test_autograd_function_uses_the_adjoint():
    from paper_1510_03816_amd.autograd import shoot
    pr = inputs.config_sphere3d(400, kernel=lm.GAUSS, sigma=0.3)
    prm = lm.make_params(3, lm.GAUSS, pr.sigma)
    q0 = dev(pr.X).requires_grad_(True)
    p0 = dev(pr.p_bench()).requires_grad_(True)
    q1, p1 = shoot(q0, p0, prm, 1.0, 15, 5)
    Yt = dev(pr.Y)
    loss = ((q1 - Yt) ** 2).sum() + (p1 ** 2).sum()
    loss.backward()
    gq1 = 2.0 * (host(q1.detach()) - pr.Y)
    gp1 = 2.0 * host(p1.detach())
    oq, op = oracle.shoot_adjoint(pr.X, pr.p_bench(), gq1, gp1, 1, pr.sigma, 15)
    assert rel_err(host(q0.grad), oq) <= 1e-10 and rel_err(host(p0.grad), op) <= 1e-10


# ------------------------------------------------------------------ gradient-based matching


@pytest.mark.parametrize("kernel,gtol,tol", [(lm.CONON, 1e-9, 1e-8), (lm.GAUSS, 1e-5, 1e-4)])
def test_lbfgs_minimiser_has_zero_oracle_gradient(kernel, gtol, tol):
    """The GPU optimiser's result is checked with the oracle's gradient (an independent
    evaluation), and against the optimality condition of the continuous problem, under
    which the final momenta equal -lam (q(1) - Y) (up to the RK4 error).  The Gaussian
    kernel matrix is far worse conditioned, so its bar is looser."""
    pr = inputs.config_sphere3d(200, kernel=kernel, sigma=0.3)
    prm = lm.make_params(3, kernel, pr.sigma)
    p0 = torch.zeros((3, 200), dtype=torch.float64, device=DEV)
    st, info = lm.lm_lbfgs_match(prm, dev(pr.X), dev(pr.Y), p0, lam=100.0, steps=20, gtol=gtol, max_iter=1000,
                                 history=16)
    print("lbfgs kernel %d: %d its, %d evals, E %.6g, |g| %.2e, resid %.2e" % (
        kernel, info.iters, info.evals, info.E, info.gnorm_inf, info.resid_inf))
    assert st == 0
    E0, g0 = oracle.energy_and_grad(pr.X, pr.Y, np.zeros_like(pr.X), kernel, pr.sigma, 100.0, 20)
    E, g = oracle.energy_and_grad(pr.X, pr.Y, host(p0), kernel, pr.sigma, 100.0, 20)
    assert E == pytest.approx(info.E, rel=1e-10)
    assert np.max(np.abs(g)) <= tol * np.max(np.abs(g0))
    q1, p1 = oracle.shoot(pr.X, host(p0), kernel, pr.sigma, 20)
    print("optimality: |p(1) + lam (q(1) - Y)| / |p(1)| = %.2e" % rel_err(p1, -100.0 * (q1 - pr.Y)))
    if kernel == lm.CONON:   # converged to 1e-9: the condition holds to the RK4 error
        assert rel_err(p1, -100.0 * (q1 - pr.Y)) <= 1e-4


def test_lbfgs_least_squares_reaches_exact_match():
    """reg = 0 leaves the least-squares shooting objective; its zero is an exact match."""
    pr = inputs.config_circle_ellipse(64)
    prm = lm.make_params(2, lm.CONON, pr.sigma)
    p0 = torch.zeros((2, 64), dtype=torch.float64, device=DEV)
    st, info = lm.lm_lbfgs_match(prm, dev(pr.X), dev(pr.Y), p0, lam=1.0, reg=0.0, steps=pr.steps, gtol=0.0,
                                 match_tol=1e-6, max_iter=2000, history=16)
    print("least squares: %d its, %d evals, resid %.2e" % (info.iters, info.evals, info.resid_inf))
    assert st == 0 and info.resid_inf < 1e-6
    q1, _ = oracle.shoot(pr.X, host(p0), 0, pr.sigma, pr.steps)
    assert np.max(np.abs(q1 - pr.Y)) < 1.1e-6
