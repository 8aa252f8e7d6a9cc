"""FP64 CPU oracle of geodesic landmark shooting (arXiv 1510.03816).  TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library never loads it; the two share no code.

``lm_oracle.c`` is the oracle proper (plain C, FP64, OpenMP over the target index only);
this module builds it with gcc and wraps it with ctypes.  ``mini.py`` is a small NumPy
transcription used to cross-check the C code on tiny inputs.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lm_oracle.c")
LIB = os.path.join(HERE, "liblm_oracle.so")

OK, EINVAL, ENOTPD, ENOTCONV, EDIVERGED = 0, -1, -2, -4, -5
CONON, GAUSS = 0, 1


def build(force: bool = True) -> str:
    """Compile lm_oracle.c into liblm_oracle.so (gcc, -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        d, i, l, P = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        L.orc_num_threads.restype = i
        L.orc_num_threads.argtypes = []
        L.orc_green.restype = d
        L.orc_green.argtypes = [i, d, d]
        L.orc_green_prime.restype = d
        L.orc_green_prime.argtypes = [i, d, d]
        L.orc_rhs.restype = None
        L.orc_rhs.argtypes = [i, l, i, d, d, P, P, P, P]
        L.orc_rhs_rows.restype = None
        L.orc_rhs_rows.argtypes = [i, l, i, d, d, P, P, P, l, P, P]
        L.orc_hamiltonian.restype = d
        L.orc_hamiltonian.argtypes = [i, l, i, d, P, P]
        L.orc_shoot.restype = None
        L.orc_shoot.argtypes = [i, l, i, d, d, d, i, P, P, P, P]
        L.orc_kmatrix.restype = None
        L.orc_kmatrix.argtypes = [i, l, i, d, P, P]
        L.orc_cholesky.restype = i
        L.orc_cholesky.argtypes = [l, P]
        L.orc_cholesky_solve.restype = None
        L.orc_cholesky_solve.argtypes = [l, P, P, P]
        L.orc_feedback_match.restype = i
        L.orc_feedback_match.argtypes = [i, l, i, d, d, P, P, d, d, i, i, i, P, P,
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(d),
                                         ctypes.POINTER(d), P, i]
        L.orc_rhs_vjp.restype = None
        L.orc_rhs_vjp.argtypes = [i, l, i, d, d, P, P, P, P, P, P]
        L.orc_shoot_adjoint.restype = None
        L.orc_shoot_adjoint.argtypes = [i, l, i, d, d, d, i, P, P, P, P, P, P]
        L.orc_velocity.restype = None
        L.orc_velocity.argtypes = [i, l, l, i, d, P, P, P, P]
        L.orc_flow_points.restype = None
        L.orc_flow_points.argtypes = [i, l, l, i, d, d, d, i, P, P, P, P, P, P]
        _lib = L
    return _lib


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return lib().orc_num_threads()


def green(kernel: int, sigma: float, r: float) -> float:
    return lib().orc_green(kernel, sigma, r)


def green_prime(kernel: int, sigma: float, r: float) -> float:
    return lib().orc_green_prime(kernel, sigma, r)


def rhs(q, p, kernel: int, sigma: float, tau: float = 0.0):
    """(dq/dt, dp/dt) of the N-particle system at state (q, p), both (dim, n)."""
    q, p = _c(q), _c(p)
    dim, n = q.shape
    dq, dp = np.empty_like(q), np.empty_like(p)
    lib().orc_rhs(dim, n, kernel, sigma, tau, _ptr(q), _ptr(p), _ptr(dq), _ptr(dp))
    return dq, dp


def rhs_rows(q, p, idx, kernel: int, sigma: float, tau: float = 0.0):
    """Rows idx of the right-hand side: returns (dq, dp) of shape (dim, len(idx))."""
    q, p = _c(q), _c(p)
    dim, n = q.shape
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    dq = np.empty((dim, len(ix)))
    dp = np.empty((dim, len(ix)))
    lib().orc_rhs_rows(dim, n, kernel, sigma, tau, _ptr(q), _ptr(p), _ptr(ix), len(ix), _ptr(dq), _ptr(dp))
    return dq, dp


def hamiltonian(q, p, kernel: int, sigma: float) -> float:
    """H = 1/2 sum_ij (p_i . p_j) G_ij (the paper prints 2H)."""
    q, p = _c(q), _c(p)
    dim, n = q.shape
    return lib().orc_hamiltonian(dim, n, kernel, sigma, _ptr(q), _ptr(p))


def shoot(q0, p0, kernel: int, sigma: float, steps: int, T: float = 1.0, tau: float = 0.0):
    """Classical RK4 over [0, T] with ``steps`` steps; returns (q(T), p(T))."""
    q0, p0 = _c(q0), _c(p0)
    dim, n = q0.shape
    q1, p1 = np.empty_like(q0), np.empty_like(p0)
    lib().orc_shoot(dim, n, kernel, sigma, tau, T, steps, _ptr(q0), _ptr(p0), _ptr(q1), _ptr(p1))
    return q1, p1


def kmatrix(X, kernel: int, sigma: float) -> np.ndarray:
    X = _c(X)
    dim, n = X.shape
    K = np.empty((n, n))
    lib().orc_kmatrix(dim, n, kernel, sigma, _ptr(X), _ptr(K))
    return K


def cholesky(A) -> tuple:
    """Returns (status, L) with L lower triangular (the upper triangle is left as given)."""
    L = _c(A).copy()
    st = lib().orc_cholesky(L.shape[0], _ptr(L))
    return st, L


def cholesky_solve(L, b) -> np.ndarray:
    L, b = _c(L), _c(b)
    x = np.empty_like(b)
    lib().orc_cholesky_solve(L.shape[0], _ptr(L), _ptr(b), _ptr(x))
    return x


class MatchResult:
    def __init__(self, status, iters, resid, H, p0, q1, hist):
        self.status, self.iters, self.resid, self.H = status, iters, resid, H
        self.p0, self.q1, self.hist = p0, q1, hist

    @property
    def paper_H(self) -> float:
        """The value the paper prints as the Hamiltonian: 2H = sum_ij (p_i . p_j) G_ij."""
        return 2.0 * self.H

    def __repr__(self):
        return "MatchResult(status=%d, iters=%d, resid=%.4g, 2H=%.6g)" % (
            self.status, self.iters, self.resid, 2.0 * self.H)


def feedback_match(X, Y, kernel: int, sigma: float, h: float, tol: float, steps: int,
                   max_iter: int = 500, p0=None, tau: float = 0.0, stop_rule: int = 0,
                   hist_len: int = 1024) -> MatchResult:
    """Algorithm 1 with M = hI and p = (K(X) + tau I)^{-1} u; see lm_oracle.c."""
    X, Y = _c(X), _c(Y)
    dim, n = X.shape
    p = np.zeros_like(X) if p0 is None else _c(p0).copy()
    q1 = np.empty_like(X)
    it, r, H = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    hist = np.full(hist_len, np.nan)
    st = lib().orc_feedback_match(dim, n, kernel, sigma, tau, _ptr(X), _ptr(Y), h, tol,
                                  max_iter, steps, stop_rule, _ptr(p), _ptr(q1),
                                  ctypes.byref(it), ctypes.byref(r), ctypes.byref(H),
                                  _ptr(hist), hist_len)
    k = it.value
    return MatchResult(st, k, r.value, H.value, p, q1, hist[:min(k + 1, hist_len)])


def velocity(q, p, x, kernel: int, sigma: float) -> np.ndarray:
    """u(x) = sum_j G(|x - q_j|) p_j at the points x (dim, m)."""
    q, p, x = _c(q), _c(p), _c(x)
    dim, n = q.shape
    m = x.shape[1]
    u = np.empty_like(x)
    lib().orc_velocity(dim, n, m, kernel, sigma, _ptr(q), _ptr(p), _ptr(x), _ptr(u))
    return u


def flow_points(q0, p0, x0, kernel: int, sigma: float, steps: int, T: float = 1.0, tau: float = 0.0):
    """RK4 over [0, T] of the particles (q, p) together with passive points x carried by the
    velocity field u of equation "u"; returns (q(T), p(T), x(T)), x given as (dim, m)."""
    q0, p0, x0 = _c(q0), _c(p0), _c(x0)
    dim, n = q0.shape
    m = x0.shape[1]
    q1, p1, x1 = np.empty_like(q0), np.empty_like(p0), np.empty_like(x0)
    lib().orc_flow_points(dim, n, m, kernel, sigma, tau, T, steps, _ptr(q0), _ptr(p0), _ptr(x0),
                          _ptr(q1), _ptr(p1), _ptr(x1))
    return q1, p1, x1


def rhs_vjp(q, p, a, b, kernel: int, sigma: float, tau: float = 0.0):
    """(aq, ap) = J^T (a, b): the cotangent of (q, p) given the cotangent (a, b) of the RHS."""
    q, p, a, b = _c(q), _c(p), _c(a), _c(b)
    dim, n = q.shape
    aq, ap = np.empty_like(q), np.empty_like(p)
    lib().orc_rhs_vjp(dim, n, kernel, sigma, tau, _ptr(q), _ptr(p), _ptr(a), _ptr(b), _ptr(aq), _ptr(ap))
    return aq, ap


def shoot_adjoint(q0, p0, gq1, gp1, kernel: int, sigma: float, steps: int, T: float = 1.0, tau: float = 0.0):
    """(gq0, gp0) = J^T (gq1, gp1) for the RK4 shooting map (q0, p0) -> (q(T), p(T))."""
    q0, p0, gq1, gp1 = _c(q0), _c(p0), _c(gq1), _c(gp1)
    dim, n = q0.shape
    gq0, gp0 = np.empty_like(q0), np.empty_like(p0)
    lib().orc_shoot_adjoint(dim, n, kernel, sigma, tau, T, steps, _ptr(q0), _ptr(p0), _ptr(gq1), _ptr(gp1),
                            _ptr(gq0), _ptr(gp0))
    return gq0, gp0


def energy_and_grad(X, Y, p0, kernel: int, sigma: float, lam: float, steps: int):
    """E(p0) = 1/2 p0^T K(X) p0 + lam/2 |q(1) - Y|^2 and its gradient in p0 (the inexact
    energy with lam = 1/sigma^2 of the paper, halved)."""
    X, Y, p0 = _c(X), _c(Y), _c(p0)
    Kp, _ = rhs(X, p0, kernel, sigma)
    q1, p1 = shoot(X, p0, kernel, sigma, steps)
    r = q1 - Y
    E = 0.5 * float(np.sum(p0 * Kp)) + 0.5 * lam * float(np.sum(r * r))
    _, gp0 = shoot_adjoint(X, p0, lam * r, np.zeros_like(p0), kernel, sigma, steps)
    return E, Kp + gp0
