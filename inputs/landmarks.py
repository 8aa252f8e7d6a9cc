"""Landmark-set generators: the paper's analytic templates and the seeded synthetic workloads.

Paper templates (two-dimensional, labelled landmarks, the k-th landmark of every curve taken
at the parameter value theta_k = 2*pi*k/N, k = 0..N-1, so that landmark k of the template
corresponds to landmark k of the target):

* ``example1``  -- circle of radius 2 matched to the ellipse a=4, b=1 rotated by 45 degrees
  and shifted by one unit in x (Section "Example 1").  The printed parametrisation of the
  target lost a factor cos(theta) in its y-component; the rotation the text describes is
  restored here (the point (4 cos t, sin t) rotated clockwise by pi/4, then shifted).
* ``example2``  -- circle of radius 2 matched to the fourth-order heart curve (Section
  "Example 2", heart-curve equation).
* ``h_distance_targets`` -- the five targets of the Hamiltonian-distance figure (circles of
  radius 1 and 3, the ellipse a=1, b=4, the half-circle/half-ellipse curve and the square of
  side 4; the square is sampled at equal arc length starting at (2, 0), counter-clockwise).

Synthetic workloads (the sizes and distributions of the performance study):

* ``config_curve2d`` -- a closed curve r(theta) = 1 + sum_k a_k cos(k theta + phi_k) pushed
  through a smooth field made of Gaussian bumps (2-D, N = 4096 by default).
* ``config_sphere3d`` -- a Fibonacci lattice on the unit sphere pushed through a smooth 3-D
  field of Gaussian bumps (3-D, N = 65536 by default).
* ``config_batched`` -- many 2-D curve problems of log-uniform size.

Everything returned is float64 in component-major layout, shape (dim, n).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "thetas", "circle", "ellipse", "example1", "example2", "heart",
    "half_circle_half_ellipse", "square", "h_distance_targets", "cluster_shapes",
    "fibonacci_sphere", "Problem", "config_circle_ellipse", "config_curve2d",
    "config_sphere3d", "config_batched", "config_adjoint3d", "random_state",
    "bench_momentum", "curve_kernel_mass", "sheet_kernel_mass", "smooth_field_2d",
    "smooth_field_3d",
]


def thetas(n: int) -> np.ndarray:
    """Equispaced parameter values theta_k = 2*pi*k/n, k = 0..n-1."""
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


def circle(n: int, r: float = 1.0, center=(0.0, 0.0)) -> np.ndarray:
    t = thetas(n)
    return np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)])


def ellipse(n: int, a: float, b: float, angle: float = 0.0, shift=(0.0, 0.0)) -> np.ndarray:
    """Points (a cos t, b sin t), rotated counter-clockwise by ``angle`` then shifted."""
    t = thetas(n)
    x, y = a * np.cos(t), b * np.sin(t)
    c, s = math.cos(angle), math.sin(angle)
    return np.stack([c * x - s * y + shift[0], s * x + c * y + shift[1]])


def example1(n: int = 64):
    """(X, Y) of Example 1: circle r=2 -> ellipse (4, 1) rotated by -pi/4 and shifted +1 in x."""
    X = circle(n, 2.0)
    Y = ellipse(n, 4.0, 1.0, angle=-math.pi / 4.0, shift=(1.0, 0.0))
    return X, Y


def heart(n: int) -> np.ndarray:
    """Fourth-order heart curve of Example 2."""
    t = thetas(n)
    x = (13.0 * np.cos(t) - 5.0 * np.cos(2 * t) - 2.0 * np.cos(3 * t) - np.cos(4 * t)) / 5.0
    y = 16.0 * np.sin(t) ** 3 / 5.0
    return np.stack([x, y])


def example2(n: int = 64):
    """(X, Y) of Example 2: circle r=2 -> heart curve."""
    return circle(n, 2.0), heart(n)


def half_circle_half_ellipse(n: int) -> np.ndarray:
    """Upper half from the circle r=3, lower half from the ellipse a=3, b=1 (figure (e))."""
    t = thetas(n)
    y = np.where(np.sin(t) >= 0.0, 3.0 * np.sin(t), np.sin(t))
    return np.stack([3.0 * np.cos(t), y])


def square(n: int, side: float = 4.0) -> np.ndarray:
    """Square of the given side centred at the origin, sampled at equal arc length.

    The walk starts at (side/2, 0) and goes counter-clockwise, so landmark k sits at arc
    length k*perimeter/n from that start.
    """
    h = side / 2.0
    per = 4.0 * side
    s = np.arange(n, dtype=np.float64) * per / n
    # unfold the boundary starting at (h, 0) going up along x = h
    pts = np.empty((2, n))
    for k, sk in enumerate(s):
        u = sk
        if u < h:                       # right edge, upper half
            pts[:, k] = (h, u)
        elif u < h + side:              # top edge, right to left
            pts[:, k] = (h - (u - h), h)
        elif u < h + 2 * side:          # left edge, top to bottom
            pts[:, k] = (-h, h - (u - h - side))
        elif u < h + 3 * side:          # bottom edge, left to right
            pts[:, k] = (-h + (u - h - 2 * side), -h)
        else:                           # right edge, lower half
            pts[:, k] = (h, -h + (u - h - 3 * side))
    return pts


def h_distance_targets(n: int = 64) -> dict:
    """Targets (b)-(f) of the Hamiltonian-distance figure; the reference (a) is circle r=2."""
    return {
        "b_circle_r1": circle(n, 1.0),
        "c_circle_r3": circle(n, 3.0),
        "d_ellipse_1_4": ellipse(n, 1.0, 4.0),
        "e_half_circle_half_ellipse": half_circle_half_ellipse(n),
        "f_square_4": square(n, 4.0),
    }


def cluster_shapes(n: int = 64) -> dict:
    """Shapes of the cluster-analysis example: ellipses A (1 x 4), B (1.05 x 4), circles C, D.

    The text gives C a radius of 1, but the Hamiltonians it prints for C match a circle of
    radius 2 (the same reference as the Hamiltonian-distance figure), which is used here.
    """
    return {
        "A": ellipse(n, 1.0, 4.0),
        "B": ellipse(n, 1.05, 4.0),
        "C": circle(n, 2.0),
        "D": circle(n, 3.0),
    }


def fibonacci_sphere(n: int) -> np.ndarray:
    """Fibonacci lattice on the unit sphere: z_i = 1-(2i+1)/n, azimuth i*pi*(3-sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z])


def smooth_field_2d(X: np.ndarray, rng, nbumps=16, width=0.3, amp=0.15, box=1.3) -> np.ndarray:
    """Displacement made of ``nbumps`` Gaussian bumps, capped at ``amp`` in max norm.

    Draw order: centres U([-box, box]^2), directions psi ~ U(0, 2 pi), magnitudes U(0, amp).
    """
    c = rng.uniform(-box, box, size=(nbumps, 2))
    psi = rng.uniform(0.0, 2.0 * math.pi, size=nbumps)
    m = rng.uniform(0.0, amp, size=nbumps)
    d = np.zeros_like(X)
    for b in range(nbumps):
        r2 = (X[0] - c[b, 0]) ** 2 + (X[1] - c[b, 1]) ** 2
        env = m[b] * np.exp(-r2 / (2.0 * width * width))
        d[0] += env * math.cos(psi[b])
        d[1] += env * math.sin(psi[b])
    mx = float(np.max(np.sqrt(d[0] ** 2 + d[1] ** 2)))
    if mx > amp:
        d *= amp / mx
    return d


def smooth_field_3d(X: np.ndarray, rng, nbumps=32, width=0.4, amp=0.1) -> np.ndarray:
    """3-D displacement of ``nbumps`` Gaussian bumps, capped at ``amp`` in max norm.

    Draw order: centres (normalised standard normals), directions (normalised standard
    normals), magnitudes U(0, amp).
    """
    c = rng.standard_normal(size=(nbumps, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    u = rng.standard_normal(size=(nbumps, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    m = rng.uniform(0.0, amp, size=nbumps)
    d = np.zeros_like(X)
    for b in range(nbumps):
        r2 = sum((X[k] - c[b, k]) ** 2 for k in range(3))
        env = m[b] * np.exp(-r2 / (2.0 * width * width))
        for k in range(3):
            d[k] += env * u[b, k]
    mx = float(np.max(np.sqrt(np.sum(d * d, axis=0))))
    if mx > amp:
        d *= amp / mx
    return d


def curve_kernel_mass(n: int, length: float, sigma: float, kernel: int) -> float:
    """Approximate row sum of the kernel matrix for n points spread evenly along a curve.

    With line density lam = n/length, the sum over neighbours of exp(-|s|/sigma) is about
    2*lam*sigma and that of exp(-s^2/sigma^2) about sqrt(pi)*lam*sigma (a continuum
    estimate of the input's local density; used only to scale a momentum guess).
    """
    lam = n / length
    return 1.0 + (2.0 * lam * sigma if kernel == 0 else math.sqrt(math.pi) * lam * sigma)


def sheet_kernel_mass(n: int, area: float, sigma: float, kernel: int) -> float:
    """Same estimate for n points spread evenly over a surface of the given area."""
    rho = n / area
    return 1.0 + (2.0 * math.pi * rho * sigma * sigma if kernel == 0
                  else math.pi * rho * sigma * sigma)


def bench_momentum(X: np.ndarray, Y: np.ndarray, mass: float) -> np.ndarray:
    """Momentum guess (Y - X)/mass: a displacement scaled by the local kernel mass."""
    return (Y - X) / mass


@dataclass
class Problem:
    """One matching problem: template X, target Y (dim, n) and its kernel settings."""
    name: str
    X: np.ndarray
    Y: np.ndarray
    kernel: int          # 0 = conical exp(-r/sigma), 1 = Gaussian exp(-r^2/sigma^2)
    sigma: float
    steps: int
    h: float = 0.8
    tol: float = 1e-6
    p_mass: float = 1.0  # scale of the throughput momentum guess
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.X.shape[0]

    @property
    def n(self) -> int:
        return self.X.shape[1]

    def p_bench(self) -> np.ndarray:
        return bench_momentum(self.X, self.Y, self.p_mass)


def config_circle_ellipse(n: int = 64) -> Problem:
    """Unit circle -> ellipse with semi-axes 1.3 and 0.8 at the same angles (2-D, conical)."""
    X = circle(n, 1.0)
    Y = ellipse(n, 1.3, 0.8)
    return Problem("circle_ellipse_n%d" % n, X, Y, kernel=0, sigma=0.5, steps=100,
                   p_mass=curve_kernel_mass(n, 2 * math.pi, 0.5, 0))


def _curve2d(n: int, rng):
    a = rng.uniform(-0.05, 0.05, size=8)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=8)
    t = thetas(n)
    r = 1.0 + sum(a[k] * np.cos((k + 1) * t + ph[k]) for k in range(8))
    X = np.stack([r * np.cos(t), r * np.sin(t)])
    Y = X + smooth_field_2d(X, rng)
    return X, Y


def config_curve2d(n: int = 4096, seed=2, sigma: float = 0.1, steps: int = 200,
                   kernel: int = 0) -> Problem:
    """Seeded closed curve and its smoothly displaced copy (2-D, conical sigma=0.1)."""
    rng = np.random.default_rng(seed)
    X, Y = _curve2d(n, rng)
    return Problem("curve2d_n%d" % n, X, Y, kernel=kernel, sigma=sigma, steps=steps,
                   p_mass=curve_kernel_mass(n, 2 * math.pi, sigma, kernel))


def config_sphere3d(n: int = 65536, seed=3, kernel: int = 0, sigma: float = 0.05,
                    steps: int = 100) -> Problem:
    """Fibonacci sphere and its smoothly displaced copy (3-D, sigma=0.05)."""
    rng = np.random.default_rng(seed)
    X = fibonacci_sphere(n)
    Y = X + smooth_field_3d(X, rng)
    return Problem("sphere3d_n%d_%s" % (n, "conon" if kernel == 0 else "gauss"), X, Y,
                   kernel=kernel, sigma=sigma, steps=steps,
                   p_mass=sheet_kernel_mass(n, 4 * math.pi, sigma, kernel))


def config_adjoint3d(n: int = 16384, seed=5, sigma: float = 0.1, steps: int = 100) -> Problem:
    """Fibonacci sphere target problem for the differentiation workload (Gaussian sigma=0.1).

    ``extra['fd_idx']`` holds 32 particle indices drawn from a separate stream for
    finite-difference checks.
    """
    pr = config_sphere3d(n, seed=seed, kernel=1, sigma=sigma, steps=steps)
    pr.name = "adjoint3d_n%d" % n
    rng = np.random.default_rng([seed, 1])
    pr.extra["fd_idx"] = np.sort(rng.choice(n, size=min(32, n), replace=False))
    pr.extra["lam"] = 100.0
    pr.extra["ckpt_every"] = 10
    return pr


def config_batched(count: int = 256, seed: int = 4, nmin: int = 32, nmax: int = 4096,
                   steps: int = 100):
    """Many independent 2-D curve problems with N_b log-uniform in [nmin, nmax].

    Returns (sizes, offsets, X, Y): X and Y are (2, sum N_b), problem b occupies columns
    offsets[b]..offsets[b+1]-1.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    X = np.empty((2, int(offs[-1])))
    Y = np.empty_like(X)
    for b in range(count):
        xb, yb = _curve2d(int(sizes[b]), np.random.default_rng([seed, b]))
        X[:, offs[b]:offs[b + 1]] = xb
        Y[:, offs[b]:offs[b + 1]] = yb
    return sizes, offs, X, Y


def random_state(n: int, dim: int, seed, box: float = 1.0, pscale: float = 0.1):
    """Uniform positions in [-box, box]^dim and normal momenta of scale ``pscale``."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(-box, box, size=(dim, n))
    p = pscale * rng.standard_normal(size=(dim, n))
    return q, p
