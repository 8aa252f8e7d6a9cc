"""Pins of the FP64 oracle against the numbers the paper prints (no GPU).

Fixtures under tests/golden/ hold the printed values with their citations.  The readings
that make them reproduce (the u-space momentum update, the maximum norm, tolerance 1e-3 for
the metric grids, 2H as the printed Hamiltonian, the restored Example 1 target, h = 0.8 for
the Hamiltonian-distance figure) are listed in the design notes.
"""

import math

import numpy as np
import pytest

import inputs
from _golden import paper_values, table2, table3

PV = paper_values()
STEPS = 50          # RK4 steps per shoot; the paper does not state its step count


def test_example1_iterations_residual_and_hamiltonian(orc):
    X, Y = inputs.example1(64)
    res = orc.feedback_match(X, Y, 0, 1.0, 0.3, 1e-3, STEPS)
    assert res.status == 0
    assert res.iters == PV["example1_iters"]
    assert float("%.1e" % res.resid) == PV["example1_resid"]       # printed to 2 digits
    assert res.paper_H == pytest.approx(PV["example1_H"], rel=1e-4)


def test_example1_literal_target_does_not_reproduce(orc):
    """The printed target formula without cos(theta) in y gives a different count, which is
    why the restored rotation is the reading used."""
    t = inputs.thetas(64)
    c = math.cos(math.pi / 4)
    Y = np.stack([4 * c * np.cos(t) + c * np.sin(t) + 1.0, c * np.sin(t) - 4 * c])
    res = orc.feedback_match(inputs.circle(64, 2.0), Y, 0, 1.0, 0.3, 1e-3, STEPS)
    assert res.iters != PV["example1_iters"]


@pytest.mark.parametrize("h,want", table2())
def test_table2_search_length(orc, h, want):
    X, Y = inputs.example2(64)
    res = orc.feedback_match(X, Y, 0, 1.0, h, 1e-3, STEPS, max_iter=500)
    if want is None:
        assert res.status == -5                       # blows up: NaN
    elif h == 0.2:
        # the recomputed residual at 82 iterations is 9.98e-4, a hair under the tolerance;
        # the printed 83 is within one iteration
        assert res.status == 0 and abs(res.iters - want) <= 1
    else:
        assert res.status == 0 and res.iters == want
    if h == 0.8:
        assert res.paper_H == pytest.approx(PV["example2_H"], rel=1e-4)


def test_table2_p_space_update_diverges(orc):
    """Updating p by h*e directly (no K^{-1}) does not reproduce the table: at h = 0.3 on
    Example 1 it blows up, which pins the u-space reading p <- p + h K^{-1} e."""
    X, Y = inputs.example1(64)
    p = np.zeros_like(X)
    for _ in range(60):
        q1, _ = orc.shoot(X, p, 0, 1.0, STEPS)
        e = Y - q1
        if not np.all(np.isfinite(e)):
            break
        p = p + 0.3 * e
    assert not np.all(np.isfinite(e)) or np.max(np.abs(e)) > 1.0


T3 = table3()
T3_CASES = [(g, a2, j, h) for g in "abcd" for (a2, _) in T3[g]["rows"]
            for j, h in enumerate([0.2, 0.4, 0.6, 0.8, 1.0])]


@pytest.mark.parametrize("grid,a2,col,h", T3_CASES)
def test_table3_metric_grid(orc, grid, a2, col, h):
    g = T3[grid]
    want = dict(g["rows"])[a2][col]
    X, Y = inputs.example2(g["n"])
    res = orc.feedback_match(X, Y, g["kernel"], math.sqrt(a2), h, 1e-3, 20, max_iter=500)
    if grid == "d" and a2 == 0.2 and h == 1.0:
        # the one cell that does not reproduce: the paper marks it x, the recomputation
        # converges in 14 iterations
        assert res.status == 0 and res.iters == 14
    elif want is None:
        assert res.status != 0
    else:
        assert res.status == 0 and res.iters == want


def test_hamiltonian_distance_figure(orc):
    C = inputs.circle(64, 2.0)
    got = {}
    for key, Yt in inputs.h_distance_targets(64).items():
        res = orc.feedback_match(C, Yt, 0, 1.0, 0.8, 1e-3, STEPS)
        assert res.status == 0
        got[key] = res.paper_H
        assert res.paper_H == pytest.approx(PV["hdist_" + key], rel=2e-4)
    # the ordering the text states: H(af) < H(ab) < H(ae) < H(ac) < H(ad)
    order = ["f_square_4", "b_circle_r1", "e_half_circle_half_ellipse", "c_circle_r3", "d_ellipse_1_4"]
    assert all(got[a] < got[b] for a, b in zip(order, order[1:]))


def test_cluster_analysis_hamiltonians(orc):
    sh = inputs.cluster_shapes(64)
    for pair, rel in [("CD", 2e-4), ("CA", 2e-4), ("CB", 2e-4), ("DA", 1e-3), ("DB", 1e-3), ("AB", 3e-2)]:
        res = orc.feedback_match(sh[pair[0]], sh[pair[1]], 0, 1.0, 0.8, 1e-3, STEPS)
        assert res.status == 0
        assert res.paper_H == pytest.approx(PV["H_" + pair], rel=rel)


def test_reference_target_asymmetry(orc):
    E, C3 = inputs.half_circle_half_ellipse(64), inputs.circle(64, 3.0)
    ec = orc.feedback_match(E, C3, 0, 1.0, 0.8, 1e-3, STEPS).paper_H
    ce = orc.feedback_match(C3, E, 0, 1.0, 0.8, 1e-3, STEPS).paper_H
    assert ec == pytest.approx(PV["H_ec"], rel=2e-4)
    assert ce == pytest.approx(PV["H_ce"], rel=5e-4)
    assert ec != ce


def test_iso_invariance_of_matched_hamiltonian(orc):
    """Table 4: H(G(A), G(B)) - H(A, B) is at rounding level for isometries G."""
    A = inputs.circle(64, 2.0)
    B = inputs.half_circle_half_ellipse(64)
    H0 = orc.feedback_match(A, B, 0, 1.0, 0.8, 1e-3, STEPS).H
    a = math.pi / 3
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    F = np.array([[1.0, 0.0], [0.0, -1.0]])
    t = np.array([[0.5], [0.5]])
    for GA, GB in [(R @ A, R @ B), (A + t, B + t), (F @ A, F @ B)]:
        H1 = orc.feedback_match(GA, GB, 0, 1.0, 0.8, 1e-3, STEPS).H
        assert abs(2 * (H1 - H0)) < 1e-11 * abs(H0)


@pytest.mark.parametrize("t", [0.2, 0.4, 0.6, 0.8])
def test_example2_phase_hamiltonians(orc, t):
    """The Example 2 figure prints an H for every intermediate phase.  Reading: the phase at
    time t is the landmark set q(t) of the circle -> heart match, and its H is that of the
    momenta Algorithm 1 (h = 0.8, tol 1e-3) finds when that phase is the target; these
    reproduce the printed values to 1e-4 (the exact geodesic segment would give t^2 times
    the t = 1 value, 0.3-0.1% off)."""
    X, Y = inputs.example2(64)
    full = orc.feedback_match(X, Y, 0, 1.0, 0.8, 1e-3, STEPS)
    It, _ = orc.shoot(X, full.p0, 0, 1.0, STEPS, T=t)
    res = orc.feedback_match(X, It, 0, 1.0, 0.8, 1e-3, STEPS)
    assert res.status == 0
    assert res.paper_H == pytest.approx(PV["example2_phase_H_%.1f" % t], rel=2e-4)
    assert abs(res.paper_H - t * t * full.paper_H) > abs(res.paper_H - PV["example2_phase_H_%.1f" % t])


def test_prediction_experiment(orc):
    """Section "The prediction ability of Algorithm 1": match the circle to the t = 0.6 phase,
    continue the flow of the momenta found to t = 1 and compare with the heart.  The momenta
    that carry the template to the phase in unit time, continued to t = 1/0.6, give the
    flow of the paper's reading (momenta reaching the phase at t = 0.6, continued to t = 1)
    by the exact time rescaling of the system.  The prediction lands on the heart to within
    the matching tolerance (1.4e-3 against the 1e-3 of the matches)."""
    X, Y = inputs.example2(64)
    full = orc.feedback_match(X, Y, 0, 1.0, 0.8, 1e-3, STEPS)
    I06, _ = orc.shoot(X, full.p0, 0, 1.0, STEPS, T=0.6)
    res = orc.feedback_match(X, I06, 0, 1.0, 0.8, 1e-3, STEPS)
    pred, _ = orc.shoot(X, res.p0, 0, 1.0, STEPS, T=1.0 / 0.6)
    err = np.max(np.abs(pred - Y))
    assert err < 2e-3
    # without the continuation the match stops at the phase, far from the heart
    assert np.max(np.abs(I06 - Y)) > 100 * err
