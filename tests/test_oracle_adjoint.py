"""Pins of the oracle's reverse mode (adjoint of the shooting map) -- no GPU.

The vector-Jacobian products are checked against central finite differences of the forward
oracle (a dot-product test <(a, b), J v> = <J^T (a, b), v> for random directions v), and the
energy gradient against the closed form at p0 = 0, where the flow is at rest and its
linearisation is q(1) = X + K(X) dp exactly.
"""

import numpy as np
import pytest

import inputs

KERNELS = [0, 1]


def _dirs(shape, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) for _ in range(4)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("tau", [0.0, 0.3])
def test_rhs_vjp_against_finite_differences(orc, kernel, dim, tau):
    q, p = inputs.random_state(7, dim, seed=[30, dim, kernel], pscale=0.4)
    a, b, dq, dp = _dirs(q.shape, [31, dim])
    sigma, eps = 0.45, 1e-6
    fq1, fp1 = orc.rhs(q + eps * dq, p + eps * dp, kernel, sigma, tau)
    fq0, fp0 = orc.rhs(q - eps * dq, p - eps * dp, kernel, sigma, tau)
    lhs = (np.sum(a * (fq1 - fq0)) + np.sum(b * (fp1 - fp0))) / (2 * eps)
    aq, ap = orc.rhs_vjp(q, p, a, b, kernel, sigma, tau)
    rhs = np.sum(aq * dq) + np.sum(ap * dp)
    assert rhs == pytest.approx(lhs, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dim", [2, 3])
def test_shoot_adjoint_against_finite_differences(orc, kernel, dim):
    q, p = inputs.random_state(6, dim, seed=[32, dim], pscale=0.3)
    gq, gp, dq, dp = _dirs(q.shape, [33, dim])
    sigma, eps, steps = 0.5, 1e-6, 12
    a1, b1 = orc.shoot(q + eps * dq, p + eps * dp, kernel, sigma, steps, T=0.9, tau=0.1)
    a0, b0 = orc.shoot(q - eps * dq, p - eps * dp, kernel, sigma, steps, T=0.9, tau=0.1)
    lhs = (np.sum(gq * (a1 - a0)) + np.sum(gp * (b1 - b0))) / (2 * eps)
    gq0, gp0 = orc.shoot_adjoint(q, p, gq, gp, kernel, sigma, steps, T=0.9, tau=0.1)
    rhs = np.sum(gq0 * dq) + np.sum(gp0 * dp)
    assert rhs == pytest.approx(lhs, rel=1e-7, abs=1e-9)


def test_adjoint_of_single_particle_is_transpose_of_straight_line(orc):
    """One particle moves as q(1) = q0 + (1 + tau) p0 with p constant, so J^T is explicit."""
    q0 = np.array([[0.2], [-0.4]])
    p0 = np.array([[0.5], [0.1]])
    gq1 = np.array([[1.5], [-2.0]])
    gp1 = np.array([[0.3], [0.7]])
    gq0, gp0 = orc.shoot_adjoint(q0, p0, gq1, gp1, 0, 0.3, 9, tau=0.25)
    assert np.allclose(gq0, gq1, atol=1e-14)
    assert np.allclose(gp0, 1.25 * gq1 + gp1, atol=1e-14)


@pytest.mark.parametrize("kernel", KERNELS)
def test_energy_gradient_at_rest_is_lam_K_times_residual(orc, kernel):
    pr = inputs.config_sphere3d(40, kernel=kernel, sigma=0.4)
    lam = 100.0
    E, g = orc.energy_and_grad(pr.X, pr.Y, np.zeros_like(pr.X), kernel, pr.sigma, lam, 10)
    K = orc.kmatrix(pr.X, kernel, pr.sigma)
    want = lam * (K @ (pr.X - pr.Y).T).T
    assert np.allclose(g, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    assert E == pytest.approx(0.5 * lam * np.sum((pr.X - pr.Y) ** 2), rel=1e-14)


@pytest.mark.parametrize("kernel", KERNELS)
def test_energy_gradient_against_finite_differences(orc, kernel):
    pr = inputs.config_sphere3d(30, kernel=kernel, sigma=0.4)
    p = 0.05 * np.random.default_rng(34).standard_normal(pr.X.shape)
    E, g = orc.energy_and_grad(pr.X, pr.Y, p, kernel, pr.sigma, 100.0, 10)
    for (c, i) in [(0, 3), (1, 17), (2, 29)]:
        e = np.zeros_like(p)
        e[c, i] = 1e-6
        Ep, _ = orc.energy_and_grad(pr.X, pr.Y, p + e, kernel, pr.sigma, 100.0, 10)
        Em, _ = orc.energy_and_grad(pr.X, pr.Y, p - e, kernel, pr.sigma, 100.0, 10)
        assert g[c, i] == pytest.approx((Ep - Em) / 2e-6, rel=1e-6)
