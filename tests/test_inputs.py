"""The seeded input generators: shapes, determinism and the properties their recipes state."""

import numpy as np

import inputs


def test_paper_templates_shapes():
    X, Y = inputs.example1(64)
    assert X.shape == Y.shape == (2, 64)
    assert np.allclose(np.hypot(X[0], X[1]), 2.0)
    # target: ellipse (4, 1) rotated by -45 degrees about the origin, then shifted by +1 in x
    c = np.cos(np.pi / 4)
    u, v = Y[0] - 1.0, Y[1]
    a, b = c * u - c * v, c * u + c * v          # undo the rotation
    assert np.allclose((a / 4) ** 2 + b ** 2, 1.0)
    H = inputs.heart(64)
    assert H.shape == (2, 64) and np.allclose(H[:, 0], [1.0, 0.0])
    S = inputs.square(64)
    assert np.allclose(np.max(np.abs(S), axis=0), 2.0)
    assert np.allclose(S[:, 0], [2.0, 0.0])
    d = np.diff(np.concatenate([S, S[:, :1]], axis=1), axis=1)
    assert np.allclose(np.abs(d).sum(axis=0), 0.25)   # equal arc length 16/64


def test_fibonacci_sphere_on_unit_sphere():
    X = inputs.fibonacci_sphere(1000)
    assert np.allclose(np.sum(X * X, axis=0), 1.0)
    assert abs(X.mean(axis=1)).max() < 2e-3


def test_workloads_are_seeded_and_capped():
    a = inputs.config_curve2d(512)
    b = inputs.config_curve2d(512)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.Y, b.Y)
    assert np.max(np.hypot(*(a.Y - a.X))) <= 0.15 + 1e-15
    s = inputs.config_sphere3d(2048)
    assert s.X.shape == (3, 2048)
    assert np.max(np.sqrt(np.sum((s.Y - s.X) ** 2, axis=0))) <= 0.1 + 1e-15
    sizes, offs, X, Y = inputs.config_batched(count=16)
    assert sizes.min() >= 32 and sizes.max() <= 4096 and offs[-1] == X.shape[1] == sizes.sum()
    c = inputs.config_adjoint3d(1024)
    assert len(c.extra["fd_idx"]) == 32 and len(set(c.extra["fd_idx"])) == 32
