"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than its own formulas: Hamilton's
equations of the discrete Hamiltonian, closed-form solutions, conservation laws, exact
symmetries of the N-particle system and library linear algebra.  A dropped term, a wrong
sign or a transposed index in the oracle fails at least one of them.
"""

import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import inputs
from oracle import mini

KERNELS = [0, 1]


def _rand(n, dim, seed, box=1.0, pscale=0.3):
    return inputs.random_state(n, dim, seed, box=box, pscale=pscale)


# ---------------------------------------------------------------- Green's functions


@pytest.mark.parametrize("kernel", KERNELS)
def test_green_special_values_and_derivative(orc, kernel):
    sigma = 0.37
    assert orc.green(kernel, sigma, 0.0) == 1.0            # normalised: G(0) = 1
    assert orc.green(kernel, sigma, sigma) == pytest.approx(math.exp(-1.0), rel=1e-15)
    for r in [0.05, 0.3, 1.0, 2.5]:
        eps = 1e-6
        fd = (orc.green(kernel, sigma, r + eps) - orc.green(kernel, sigma, r - eps)) / (2 * eps)
        assert orc.green_prime(kernel, sigma, r) == pytest.approx(fd, rel=1e-8, abs=1e-12)
    # monotone decreasing (both kernels are positive-definite radial functions)
    rs = np.linspace(0, 3, 50)
    g = [orc.green(kernel, sigma, r) for r in rs]
    assert all(a > b for a, b in zip(g, g[1:]))


# ---------------------------------------------------------------- the N-particle system


def test_hamiltonian_two_particles_by_hand(orc):
    q = np.array([[0.1, 0.7], [-0.2, 0.3]])
    p = np.array([[0.5, -0.25], [0.125, 0.75]])
    r = math.hypot(0.6, 0.5)
    for kernel, G in [(0, math.exp(-r / 0.4)), (1, math.exp(-(r / 0.4) ** 2))]:
        p1p2 = 0.5 * -0.25 + 0.125 * 0.75
        want = 0.5 * (0.5 ** 2 + 0.125 ** 2 + 0.25 ** 2 + 0.75 ** 2) + p1p2 * G
        assert orc.hamiltonian(q, p, kernel, 0.4) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("tau", [0.0, 0.3])
def test_rhs_obeys_hamiltons_equations(orc, kernel, dim, tau):
    """dq/dt = dH/dp, dp/dt = -dH/dq (equation "charsham", discrete form), by central
    differences of the Hamiltonian; the inexact system adds tau/2 sum |p_i|^2 to H."""
    n, sigma = 6, 0.45
    q, p = _rand(n, dim, seed=[11, kernel, dim])
    dq, dp = orc.rhs(q, p, kernel, sigma, tau)

    def Htau(qq, pp):
        return orc.hamiltonian(qq, pp, kernel, sigma) + 0.5 * tau * float(np.sum(pp * pp))

    eps = 1e-6
    for c in range(dim):
        for i in range(n):
            e = np.zeros_like(q)
            e[c, i] = eps
            dHdp = (Htau(q, p + e) - Htau(q, p - e)) / (2 * eps)
            dHdq = (Htau(q + e, p) - Htau(q - e, p)) / (2 * eps)
            assert dq[c, i] == pytest.approx(dHdp, rel=1e-7, abs=1e-9)
            assert dp[c, i] == pytest.approx(-dHdq, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("kernel", KERNELS)
def test_forces_sum_to_zero(orc, kernel):
    q, p = _rand(50, 3, seed=12)
    _, dp = orc.rhs(q, p, kernel, 0.3)
    assert np.max(np.abs(dp.sum(axis=1))) < 1e-14 * max(1.0, np.max(np.abs(dp)) * 50)


def test_coincident_particles_exert_no_force(orc):
    q = np.array([[0.3, 0.3, 1.0], [0.2, 0.2, -0.5]])
    p = np.array([[0.1, -0.4, 0.2], [0.3, 0.05, 0.0]])
    for kernel in KERNELS:
        dq, dp = orc.rhs(q, p, kernel, 0.5)
        assert np.all(np.isfinite(dp))
        # particles 0 and 1 see each other with G(0) = 1 in the velocity sum
        g02 = orc.green(kernel, 0.5, math.hypot(0.7, 0.7))
        assert dq[:, 0] == pytest.approx(p[:, 0] + p[:, 1] + g02 * p[:, 2], rel=1e-14)
        # the force on 0 is the force from particle 2 alone: the coincident particle 1
        # contributes nothing
        _, dp2 = orc.rhs(q[:, [0, 2]], p[:, [0, 2]], kernel, 0.5)
        assert dp[:, 0] == pytest.approx(dp2[:, 0], rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("tau", [0.0, 0.3])
@pytest.mark.parametrize("nidx", [5, 300])
def test_rhs_rows_equals_rows_of_the_full_rhs_bitwise(orc, kernel, dim, tau, nidx):
    """The sampled-rows form of the right-hand side (which every full-size comparison uses)
    returns exactly the selected rows of the full evaluation, for unsorted and repeated
    indices, the first and last rows, and coincident particles; both sides of its threaded
    branch (few rows and many)."""
    n = 150
    q, p = _rand(n, dim, seed=[31, dim, nidx])
    q[:, 7] = q[:, 99]                        # a coincident pair
    rng = np.random.default_rng([32, nidx])
    idx = np.concatenate([[n - 1, 0, 7, 99, 7], rng.integers(0, n, size=nidx - 5)])[:nidx]
    assert len(set(idx.tolist())) < nidx      # repeats, and not sorted
    assert not np.all(np.diff(idx) >= 0)
    dq, dp = orc.rhs(q, p, kernel, 0.4, tau)
    rq, rp = orc.rhs_rows(q, p, idx, kernel, 0.4, tau)
    assert rq.shape == (dim, nidx) and rp.shape == (dim, nidx)
    assert np.array_equal(rq, dq[:, idx])
    assert np.array_equal(rp, dp[:, idx])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n,dim", [(1, 2), (2, 2), (3, 3), (7, 2), (20, 3)])
def test_c_oracle_matches_numpy_mini(orc, kernel, n, dim):
    q, p = _rand(n, dim, seed=[13, n, dim])
    dq, dp = orc.rhs(q, p, kernel, 0.6, 0.2)
    mq, mp = mini.rhs(q, p, kernel, 0.6, 0.2)
    assert np.allclose(dq, mq, rtol=1e-13, atol=1e-15)
    assert np.allclose(dp, mp, rtol=1e-13, atol=1e-15)
    assert orc.hamiltonian(q, p, kernel, 0.6) == pytest.approx(mini.hamiltonian(q, p, kernel, 0.6), rel=1e-13)
    q1, p1 = orc.shoot(q, p, kernel, 0.6, 10, tau=0.2)
    m1, n1 = mini.shoot(q, p, kernel, 0.6, 10, tau=0.2)
    assert np.allclose(q1, m1, rtol=1e-12, atol=1e-14)
    assert np.allclose(p1, n1, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- the shooting map


@pytest.mark.parametrize("tau", [0.0, 0.5])
def test_single_particle_moves_in_a_straight_line(orc, tau):
    q0 = np.array([[0.3], [-1.2], [2.0]])
    p0 = np.array([[0.7], [0.1], [-0.4]])
    for kernel in KERNELS:
        q1, p1 = orc.shoot(q0, p0, kernel, 0.2, 13, T=1.0, tau=tau)
        assert np.allclose(q1, q0 + (1.0 + tau) * p0, rtol=0, atol=1e-14)   # 13 roundings
        assert np.array_equal(p1, p0)


def _two_body_conon_exact(Q0, P0, sigma, t):
    """Head-on separating pair at +-Q/2 with momenta +-P (outward), conon kernel.

    H = P^2 (1 - exp(-Q/sigma)) is conserved; with w = sqrt(1 - exp(-Q/sigma)) the reduced
    equation is dw/dt = sqrt(H) (1 - w^2)/sigma, so w = tanh(atanh(w0) + sqrt(H) t/sigma) and
    Q = 2 sigma ln cosh(atanh(w0) + sqrt(H) t/sigma), P = sqrt(H)/w.
    """
    H = P0 ** 2 * (1.0 - math.exp(-Q0 / sigma))
    w0 = math.sqrt(1.0 - math.exp(-Q0 / sigma))
    a = math.atanh(w0) + math.sqrt(H) * t / sigma
    return 2.0 * sigma * math.log(math.cosh(a)), math.sqrt(H) / math.tanh(a)


def _two_body_state(Q0, P0):
    q = np.array([[Q0 / 2, -Q0 / 2], [0.0, 0.0]])
    p = np.array([[P0, -P0], [0.0, 0.0]])
    return q, p


def test_two_body_conon_closed_form_fourth_order(orc):
    Q0, P0, sigma = 0.5, 0.3, 0.5
    Qx, Px = _two_body_conon_exact(Q0, P0, sigma, 1.0)
    q, p = _two_body_state(Q0, P0)
    errs = []
    for n in [10, 20, 40]:
        q1, p1 = orc.shoot(q, p, 0, sigma, n)
        errs.append(abs((q1[0, 0] - q1[0, 1]) - Qx) + abs(p1[0, 0] - Px))
        assert abs(q1[1]).max() == 0.0 and abs(p1[1]).max() == 0.0
    assert 12.0 < errs[0] / errs[1] < 20.0
    assert 12.0 < errs[1] / errs[2] < 20.0
    q1, p1 = orc.shoot(q, p, 0, sigma, 400)
    assert (q1[0, 0] - q1[0, 1]) == pytest.approx(Qx, rel=1e-11)
    assert p1[0, 0] == pytest.approx(Px, rel=1e-11)


def test_two_body_gaussian_by_quadrature(orc):
    """Same pair with the Gaussian kernel: H = P^2 (1 - exp(-Q^2/s^2)) and
    dQ/dt = 2 sqrt(H) sqrt(1 - exp(-Q^2/s^2)), so t = int_{Q0}^{Q(t)} dQ / that."""
    Q0, P0, sigma = 0.4, 0.25, 0.5
    q, p = _two_body_state(Q0, P0)
    q1, p1 = orc.shoot(q, p, 1, sigma, 400)
    Q1 = q1[0, 0] - q1[0, 1]
    H = P0 ** 2 * (1 - math.exp(-(Q0 / sigma) ** 2))
    t, _ = scipy.integrate.quad(lambda Q: 1.0 / (2 * math.sqrt(H) * math.sqrt(-math.expm1(-(Q / sigma) ** 2))),
                                Q0, Q1, epsabs=1e-14, epsrel=1e-13)
    assert t == pytest.approx(1.0, rel=1e-10)
    assert p1[0, 0] ** 2 * (1 - math.exp(-(Q1 / sigma) ** 2)) == pytest.approx(H, rel=1e-10)


@pytest.mark.parametrize("kernel", KERNELS)
def test_mirror_symmetric_pair_stays_symmetric(orc, kernel):
    q = np.array([[0.4, -0.4], [0.1, 0.1]])
    p = np.array([[-0.3, 0.3], [0.2, 0.2]])     # collide obliquely, mirrored about x = 0
    q1, p1 = orc.shoot(q, p, kernel, 0.5, 50)
    assert q1[0, 0] == pytest.approx(-q1[0, 1], abs=1e-15)
    assert q1[1, 0] == pytest.approx(q1[1, 1], abs=1e-15)
    assert p1[0, 0] == pytest.approx(-p1[0, 1], abs=1e-15)
    assert p1[1, 0] == pytest.approx(p1[1, 1], abs=1e-15)


@pytest.mark.parametrize("kernel", KERNELS)
def test_total_momentum_is_conserved(orc, kernel):
    q, p = _rand(30, 3, seed=14)
    q1, p1 = orc.shoot(q, p, kernel, 0.4, 20)
    assert np.max(np.abs(p1.sum(axis=1) - p.sum(axis=1))) < 1e-13


@pytest.mark.parametrize("kernel", KERNELS)
def test_energy_and_angular_momentum_drift_fourth_order(orc, kernel):
    # particles well apart and gentle momenta keep the pairs away from the conon's cusp at
    # r = 0, where the right-hand side is not smooth and RK4 loses its order
    q = 2.0 * inputs.circle(16, 1.0) + 0.1 * _rand(16, 2, seed=15)[0]
    p = 0.15 * _rand(16, 2, seed=16)[1]
    sigma = 0.5
    H0 = orc.hamiltonian(q, p, kernel, sigma)
    J0 = float(np.sum(q[0] * p[1] - q[1] * p[0]))
    dH, dJ = [], []
    for n in [5, 10, 20]:
        q1, p1 = orc.shoot(q, p, kernel, sigma, n)
        dH.append(abs(orc.hamiltonian(q1, p1, kernel, sigma) - H0))
        dJ.append(abs(float(np.sum(q1[0] * p1[1] - q1[1] * p1[0])) - J0))
    for d in (dH, dJ):
        assert 10.0 < d[0] / d[1] < 24.0 and 10.0 < d[1] / d[2] < 24.0


@pytest.mark.parametrize("kernel", KERNELS)
def test_inexact_hamiltonian_drift_fourth_order(orc, kernel):
    """The inexact system (eq. N-particle-inexact) is Hamiltonian with
    H_tau = H + tau/2 sum |p_i|^2: RK4 conserves it to fourth order."""
    q = 2.0 * inputs.circle(16, 1.0) + 0.1 * _rand(16, 2, seed=17)[0]
    p = 0.15 * _rand(16, 2, seed=18)[1]
    sigma, tau = 0.5, 0.3

    def Htau(qq, pp):
        return orc.hamiltonian(qq, pp, kernel, sigma) + 0.5 * tau * float(np.sum(pp * pp))

    H0 = Htau(q, p)
    d = []
    for n in [5, 10, 20]:
        q1, p1 = orc.shoot(q, p, kernel, sigma, n, tau=tau)
        d.append(abs(Htau(q1, p1) - H0))
    assert 10.0 < d[0] / d[1] < 24.0 and 10.0 < d[1] / d[2] < 24.0


def test_inexact_stop_rule_is_the_momentum_step(orc):
    """stop_rule 1 stops at the first k >= 1 whose last update h max|e^(k-1)| was below tol:
    the count follows from the residual history of the same iteration run by rule 0."""
    X, Y = inputs.circle(32, 1.0), inputs.ellipse(32, 1.3, 0.8)
    h, tol = 0.8, 1e-3
    full = orc.feedback_match(X, Y, 0, 0.5, h, 1e-12, 20, max_iter=40, tau=0.1)
    k_want = next(k for k in range(1, len(full.hist)) if h * full.hist[k - 1] < tol)
    res = orc.feedback_match(X, Y, 0, 0.5, h, tol, 20, max_iter=40, tau=0.1, stop_rule=1)
    assert res.status == 0 and res.iters == k_want
    assert np.array_equal(res.hist, full.hist[:k_want + 1])


def _rot3(a, b, c):
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, math.cos(c), -math.sin(c)], [0, math.sin(c), math.cos(c)]])
    return Rz @ Ry @ Rx


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_shoot_is_equivariant_under_isometries(orc, kernel, dim):
    """shoot(R X + t, R p) = (R q + t, R p) for rotations, reflections and translations."""
    q, p = _rand(12, dim, seed=[16, dim], pscale=0.4)
    q1, p1 = orc.shoot(q, p, kernel, 0.5, 20)
    if dim == 2:
        a = math.pi / 3
        mats = [np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]]),
                np.array([[1.0, 0.0], [0.0, -1.0]])]
    else:
        mats = [_rot3(0.3, -1.1, 2.0), np.diag([1.0, -1.0, 1.0])]
    shift = np.full((dim, 1), 0.5)
    for R in mats:
        qr, pr = orc.shoot(R @ q + shift, R @ p, kernel, 0.5, 20)
        assert np.allclose(qr, R @ q1 + shift, rtol=0, atol=1e-13)
        assert np.allclose(pr, R @ p1, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kernel", KERNELS)
def test_time_rescaling(orc, kernel):
    """The flow of c*p0 to t = 1 is the flow of p0 to t = c with momenta scaled by c."""
    q, p = _rand(10, 2, seed=17, pscale=0.4)
    c = 0.6
    qa, pa = orc.shoot(q, c * p, kernel, 0.5, 25, T=1.0)
    qb, pb = orc.shoot(q, p, kernel, 0.5, 25, T=c)
    assert np.allclose(qa, qb, rtol=0, atol=1e-14)
    assert np.allclose(pa, c * pb, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- linear algebra and Algorithm 1


def test_cholesky_matches_scipy(orc):
    rng = np.random.default_rng(18)
    A = rng.standard_normal((40, 40))
    A = A @ A.T + 40 * np.eye(40)
    st, L = orc.cholesky(A)
    assert st == 0
    Lref = scipy.linalg.cholesky(A, lower=True)
    assert np.allclose(np.tril(L), Lref, rtol=1e-13, atol=1e-13)
    b = rng.standard_normal(40)
    x = orc.cholesky_solve(L, b)
    assert np.allclose(x, scipy.linalg.solve(A, b, assume_a="pos"), rtol=1e-12, atol=1e-13)
    st, _ = orc.cholesky(-np.eye(3))
    assert st == -2


@pytest.mark.parametrize("kernel", KERNELS)
def test_kernel_matrix_is_positive_definite(orc, kernel):
    X = inputs.fibonacci_sphere(200)
    K = orc.kmatrix(X, kernel, 0.3)
    assert np.allclose(K, K.T, rtol=0, atol=0)
    assert np.all(np.diag(K) == 1.0)
    assert np.linalg.eigvalsh(K).min() > 0.0


@pytest.mark.parametrize("h", [0.3, 0.6])
def test_small_deformation_contracts_by_one_minus_h(orc, h):
    """At p = 0 the linearised shooting map is q(1) = X + K(X) p = X + u, so with the update
    p <- p + h K^{-1} e every residual shrinks by exactly (1 - h) to first order."""
    X = inputs.circle(32, 1.0)
    Y = X + 1e-4 * np.stack([np.sin(3 * X[1]), np.cos(2 * X[0])])
    res = orc.feedback_match(X, Y, 0, 0.5, h, 1e-12, 20, max_iter=6)
    ratios = res.hist[1:6] / res.hist[0:5]
    assert np.allclose(ratios, 1.0 - h, rtol=0, atol=2e-3)


@pytest.mark.parametrize("kernel", KERNELS)
def test_feedback_reaches_target_on_tiny_case(orc, kernel):
    X = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    Y = X + np.array([[0.05, 0.1, -0.05], [0.1, -0.05, 0.02]])
    res = orc.feedback_match(X, Y, kernel, 0.7, 0.8, 1e-10, 40, max_iter=200)
    assert res.status == 0
    q1, _ = orc.shoot(X, res.p0, kernel, 0.7, 40)
    assert np.max(np.abs(q1 - Y)) < 1e-10


def test_velocity_field_at_particles_is_particle_velocity(orc):
    q, p = _rand(25, 3, seed=19)
    for kernel in KERNELS:
        dq, _ = orc.rhs(q, p, kernel, 0.4)
        u = orc.velocity(q, p, q, kernel, 0.4)
        assert np.allclose(u, dq, rtol=1e-14, atol=1e-15)
        far = np.full((3, 2), 50.0)
        assert np.max(np.abs(orc.velocity(q, p, far, kernel, 0.4))) < 1e-40


# ---------------------------------------------------------------- flow of arbitrary points (equation "u")


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_points_at_the_particles_follow_them_bitwise(orc, kernel, dim):
    """Points placed on the particles have the particles' velocity at every stage (the
    velocity sum of a particle is the field at its position), so they follow q(t) exactly;
    the particles themselves evolve as in the plain shoot."""
    q, p = _rand(23, dim, seed=40)
    x = np.concatenate([q, q[:, :5]], axis=1)           # also repeated points
    q1, p1, x1 = orc.flow_points(q, p, x, kernel, 0.4, 17, T=0.9)
    qs, ps = orc.shoot(q, p, kernel, 0.4, 17, T=0.9)
    assert np.array_equal(q1, qs) and np.array_equal(p1, ps)
    assert np.array_equal(x1[:, :23], qs) and np.array_equal(x1[:, 23:], qs[:, :5])


def _lone_particle_conon_ahead(z0, P, sigma, t):
    """A point on the line of a lone particle (conon), z = signed distance ahead of it along
    p: dz/dt = (exp(-|z|/sigma) - 1) P.  For z > 0, sigma ln(exp(z/sigma) - 1) decreases at
    rate P; for z < 0 the distance behind grows by the mirror image."""
    if z0 > 0:
        return sigma * math.log1p(math.expm1(z0 / sigma) * math.exp(-P * t / sigma))
    return -sigma * math.log1p(math.expm1(-z0 / sigma) * math.exp(P * t / sigma))


def test_lone_particle_carries_points_on_straight_lines(orc):
    """One particle moves at constant momentum; the field it carries is parallel to p
    everywhere, so every point moves on a straight line parallel to p, and a point on the
    particle's line of motion follows the closed form of its 1-D equation."""
    sigma = 0.3
    q0 = np.array([[0.2], [-0.1], [0.4]])
    p0 = np.array([[0.6], [0.3], [-0.2]])
    P = float(np.linalg.norm(p0))
    e = p0[:, 0] / P
    zs = [0.05, 0.2, 0.7, -0.1, -0.5]
    line = np.stack([q0[:, 0] + z * e for z in zs], axis=1)
    off = q0 + np.array([[0.3, -0.2], [0.1, 0.4], [0.45, 0.25]])         # off the line
    x0 = np.concatenate([line, off], axis=1)
    for n, tol in [(20, 1e-6), (200, 1e-10)]:
        q1, p1, x1 = orc.flow_points(q0, p0, x0, 0, sigma, n, T=1.0)
        assert np.allclose(q1, q0 + p0, rtol=0, atol=1e-14) and np.array_equal(p1, p0)
        for a, z0 in enumerate(zs):
            want = q1[:, 0] + _lone_particle_conon_ahead(z0, P, sigma, 1.0) * e
            assert np.max(np.abs(x1[:, a] - want)) < tol
    # displacements parallel to p: no component across it
    d = x1 - x0
    across = d - np.outer(e, e @ d)
    assert np.max(np.abs(across)) < 1e-14


def test_lone_particle_gaussian_point_by_quadrature(orc):
    """Gaussian kernel, a point ahead on the line: dz/dt = -(1 - exp(-z^2/sigma^2)) P, so
    t = int_{z(t)}^{z0} dz / ((1 - exp(-z^2/sigma^2)) P)."""
    sigma, z0 = 0.4, 0.3
    q0 = np.array([[0.0], [0.0]])
    p0 = np.array([[0.5], [0.0]])
    x0 = np.array([[z0], [0.0]])
    _, _, x1 = orc.flow_points(q0, p0, x0, 1, sigma, 400, T=1.0)
    z1 = x1[0, 0] - 0.5
    t, _ = scipy.integrate.quad(lambda z: 1.0 / (-math.expm1(-(z / sigma) ** 2) * 0.5), z1, z0,
                                epsabs=1e-14, epsrel=1e-13)
    assert t == pytest.approx(1.0, rel=1e-10)
    assert x1[1, 0] == 0.0


@pytest.mark.parametrize("kernel", KERNELS)
def test_flow_of_points_time_rescaling(orc, kernel):
    """The points carried by c*p0 to t = 1 are those carried by p0 to t = c."""
    q, p = _rand(12, 2, seed=41, pscale=0.4)
    x = np.random.default_rng(42).uniform(-1, 1, (2, 30))
    c = 1.0 / 0.6
    _, _, xa = orc.flow_points(q, c * p, x, kernel, 0.5, 25, T=1.0)
    _, _, xb = orc.flow_points(q, p, x, kernel, 0.5, 25, T=c)
    assert np.allclose(xa, xb, rtol=0, atol=1e-14)


def test_far_points_do_not_move_and_flow_is_fourth_order(orc):
    """Points far outside the particles' reach stay put; the point flow converges at fourth
    order in the step (errors fall about 16x per halving)."""
    q, p = _rand(8, 2, seed=43, pscale=0.5)
    x = np.concatenate([np.random.default_rng(44).uniform(-1, 1, (2, 6)), np.full((2, 1), 80.0)], axis=1)
    ref = orc.flow_points(q, p, x, 0, 0.4, 640)[2]
    assert np.array_equal(ref[:, -1], x[:, -1])
    errs = [np.max(np.abs(orc.flow_points(q, p, x, 0, 0.4, n)[2] - ref)) for n in (10, 20, 40)]
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0
