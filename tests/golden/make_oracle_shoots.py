#!/usr/bin/env python3
"""Writes the stored FP64 oracle shoots of the full-size workloads (tests/golden/*.npz).

Calls only the oracle (oracle/) on inputs from inputs/: nothing here comes from the GPU
library.  Each file holds, for one workload, the sampled rows of the oracle's RK4 shoot
(q(T), p(T)) from the template X with the throughput momenta p_bench (or every row for the
2-D curve), the row indices, a sample of the inputs (so a reader can tell that the generator
still gives the same points), and the settings.

    python tests/golden/make_oracle_shoots.py [name ...]

Names (default: all but the 100-step sphere shoot, which takes over an hour on 8 cores):
  sphere3d_conon_2steps   65536 Fibonacci-sphere points, conical sigma = 0.05, 2 RK4 steps of
                          dt = 1/100 (the first two steps of the 100-step shoot)
  sphere3d_gauss_2steps   the same with the Gaussian kernel
  sphere3d_conon_100steps the whole 100-step shoot on [0, 1] (conical)
  curve2d_conon_200steps  4096-point 2-D curve, conical sigma = 0.1, 200 RK4 steps on [0, 1]
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

SAMPLE_ROWS = 4096
SAMPLE_SEED = 20151013


def sample_rows(n: int) -> np.ndarray:
    """Sorted row sample: the first and last rows plus a seeded choice of the others."""
    if n <= SAMPLE_ROWS:
        return np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(SAMPLE_SEED)
    inner = rng.choice(np.arange(1, n - 1), size=SAMPLE_ROWS - 2, replace=False)
    return np.sort(np.concatenate([[0, n - 1], inner])).astype(np.int64)


def problem(name: str):
    """(Problem, steps taken, end time T) of a stored workload."""
    if name.startswith("sphere3d"):
        kernel = 0 if "_conon_" in name else 1
        pr = inputs.config_sphere3d(65536, kernel=kernel, sigma=0.05, steps=100)
        if name.endswith("_2steps"):
            return pr, 2, 2.0 / pr.steps
        return pr, pr.steps, 1.0
    if name == "curve2d_conon_200steps":
        pr = inputs.config_curve2d(4096, kernel=0, sigma=0.1, steps=200)
        return pr, pr.steps, 1.0
    raise KeyError(name)


NAMES = ["sphere3d_conon_2steps", "sphere3d_gauss_2steps", "sphere3d_conon_100steps", "curve2d_conon_200steps"]
DEFAULT = [n for n in NAMES if n != "sphere3d_conon_100steps"]


def path(name: str) -> str:
    return os.path.join(HERE, "oracle_shoot_%s.npz" % name)


def make(name: str) -> str:
    pr, steps, T = problem(name)
    p0 = pr.p_bench()
    t0 = time.time()
    q1, p1 = oracle.shoot(pr.X, p0, pr.kernel, pr.sigma, steps, T=T)
    dt = time.time() - t0
    idx = sample_rows(pr.n)
    out = path(name)
    np.savez(out, idx=idx, q1=q1[:, idx], p1=p1[:, idx], X=pr.X[:, idx], p0=p0[:, idx],
             n=pr.n, dim=pr.dim, kernel=pr.kernel, sigma=pr.sigma, steps=steps, T=T,
             oracle_seconds=dt, oracle_threads=oracle.num_threads())
    print("%s: %d steps to T = %g in %.1f s on %d threads -> %s" % (name, steps, T, dt, oracle.num_threads(), out),
          flush=True)
    return out


if __name__ == "__main__":
    for nm in (sys.argv[1:] or DEFAULT):
        make(nm)
