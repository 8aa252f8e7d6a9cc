"""NumPy mini-oracle for tiny inputs.  TEST INFRASTRUCTURE ONLY.

An independent, vectorised transcription of the N-particle system (equation "N-particle"),
its Hamiltonian (equation "H") and a classical RK4 shoot, used to cross-check the C oracle
for small n (it builds full n x n arrays).  Same readings as lm_oracle.c: the self term is
in the velocity sum, excluded from the force sum; coincident distinct particles exert no
force.
"""

from __future__ import annotations

import numpy as np


def _pair_arrays(q):
    diff = q[:, :, None] - q[:, None, :]        # (dim, n, n): q_i - q_j
    r = np.sqrt(np.sum(diff * diff, axis=0))    # (n, n)
    return diff, r


def green(kernel: int, sigma: float, r):
    return np.exp(-r / sigma) if kernel == 0 else np.exp(-(r / sigma) ** 2)


def green_prime(kernel: int, sigma: float, r):
    if kernel == 0:
        return -np.exp(-r / sigma) / sigma
    return -2.0 * r / sigma ** 2 * np.exp(-(r / sigma) ** 2)


def rhs(q, p, kernel: int, sigma: float, tau: float = 0.0):
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    diff, r = _pair_arrays(q)
    G = green(kernel, sigma, r)
    dq = p @ G.T + tau * p                       # sum_j G_ij p_j
    pp = p.T @ p                                 # (n, n): p_i . p_j
    mask = r > 0.0                               # drops j == i and coincident pairs
    rs = np.where(mask, r, 1.0)
    coef = np.where(mask, pp * green_prime(kernel, sigma, r) / rs, 0.0)
    dp = -np.sum(coef[None, :, :] * diff, axis=2)
    return dq, dp


def hamiltonian(q, p, kernel: int, sigma: float) -> float:
    _, r = _pair_arrays(np.asarray(q, dtype=np.float64))
    p = np.asarray(p, dtype=np.float64)
    return 0.5 * float(np.sum((p.T @ p) * green(kernel, sigma, r)))


def shoot(q0, p0, kernel: int, sigma: float, steps: int, T: float = 1.0, tau: float = 0.0):
    q = np.array(q0, dtype=np.float64)
    p = np.array(p0, dtype=np.float64)
    dt = T / steps
    for _ in range(steps):
        a1, b1 = rhs(q, p, kernel, sigma, tau)
        a2, b2 = rhs(q + 0.5 * dt * a1, p + 0.5 * dt * b1, kernel, sigma, tau)
        a3, b3 = rhs(q + 0.5 * dt * a2, p + 0.5 * dt * b2, kernel, sigma, tau)
        a4, b4 = rhs(q + dt * a3, p + dt * b3, kernel, sigma, tau)
        q = q + dt / 6.0 * (a1 + 2 * a2 + 2 * a3 + a4)
        p = p + dt / 6.0 * (b1 + 2 * b2 + 2 * b3 + b4)
    return q, p
