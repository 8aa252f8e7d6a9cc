"""Batches of independent problems on the GPU, against the FP64 oracle problem by problem.

A batch is, by definition, its problems taken one at a time: the oracle of a batch is the
single-problem oracle called on every problem.  Tolerances as in test_gpu_parity.py
(normwise per problem and output array): 1e-10 in FP64, 1e-4 for the FP32 form.
"""

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


def ragged_batch(sizes, dim, seed, box=1.0, pscale=0.1):
    """Concatenated random states of the given sizes: (offs, q, p) with q, p (dim, sum)."""
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    qs, ps = [], []
    for b, n in enumerate(sizes):
        q, p = inputs.random_state(int(n), dim, [seed, b], box=box, pscale=pscale)
        qs.append(q)
        ps.append(p)
    return offs, np.concatenate(qs, axis=1), np.concatenate(ps, axis=1)


def curve_batch(count, nmax, steps=20):
    """A small batch built like the 256-problem workload (2-D curves, log-uniform sizes)."""
    sizes, offs, X, Y = inputs.config_batched(count=count, nmax=nmax, steps=steps)
    return sizes, offs, X, Y


SIZES = [1, 5, 63, 64, 65, 200, 333, 700]


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("dim,kernel,tau", [(2, lm.CONON, 0.0), (3, lm.CONON, 0.1), (2, lm.GAUSS, 0.0),
                                            (3, lm.GAUSS, 0.2)])
def test_batched_rhs_matches_oracle(dim, kernel, tau, dtype):
    offs, q, p = ragged_batch(SIZES, dim, seed=301)
    q, p = rounded(q, dtype), rounded(p, dtype)
    prm = lm.make_params(dim, kernel, 0.3, dtype=dtype, tau=tau)
    dq, dp = torch.empty_like(dev(q, dtype)), torch.empty_like(dev(q, dtype))
    lm.lm_rhs_batched(prm, offs, dev(q, dtype), dev(p, dtype), dq, dp)
    torch.cuda.synchronize()
    gq, gp = host(dq), host(dp)
    for b in range(len(SIZES)):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.rhs(q[:, s], p[:, s], kernel, 0.3, tau)
        assert rel_err(gq[:, s], oq) <= TOL[dtype], (b, rel_err(gq[:, s], oq))
        if SIZES[b] > 1:
            assert rel_err(gp[:, s], op) <= TOL[dtype], (b, rel_err(gp[:, s], op))
        else:
            assert np.all(gp[:, s] == 0.0)       # a lone particle feels no force


@pytest.mark.parametrize("split,groups", [(1, 0), (2, 0), (4, 7), (8, 256), (64, 1), (3, 1000)])
def test_batched_rhs_independent_of_launch_shape(split, groups):
    """Every split and grid size gives the oracle's answer (the source order of a split sum
    differs, so agreement is to rounding, not bitwise)."""
    offs, q, p = ragged_batch(SIZES, 2, seed=302)
    prm = lm.make_params(2, lm.CONON, 0.25)
    t = lm.lm_batch_default_tuning(offs)
    for k in range(len(t.split)):
        t.split[k] = split
    t.groups = groups
    dq, dp = torch.empty_like(dev(q)), torch.empty_like(dev(q))
    lm.lm_rhs_batched(prm, offs, dev(q), dev(p), dq, dp, tuning=t)
    torch.cuda.synchronize()
    for b in range(len(SIZES)):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.rhs(q[:, s], p[:, s], lm.CONON, 0.25)
        assert rel_err(host(dq)[:, s], oq) <= 1e-10
        if SIZES[b] > 1:
            assert rel_err(host(dp)[:, s], op) <= 1e-10


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_batched_shoot_matches_oracle(dtype):
    sizes, offs, X, Y = curve_batch(6, 400)
    p0 = np.concatenate([inputs.bench_momentum(X[:, offs[b]:offs[b + 1]], Y[:, offs[b]:offs[b + 1]],
                                               inputs.curve_kernel_mass(int(sizes[b]), 2 * np.pi, 0.1, 0))
                         for b in range(len(sizes))], axis=1)
    X, p0 = rounded(X, dtype), rounded(p0, dtype)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=dtype)
    q1, p1 = torch.empty_like(dev(X, dtype)), torch.empty_like(dev(X, dtype))
    lm.lm_shoot_batched(prm, offs, dev(X, dtype), dev(p0, dtype), 1.0, 20, q1, p1)
    torch.cuda.synchronize()
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.shoot(X[:, s], p0[:, s], lm.CONON, 0.1, 20)
        assert rel_err(host(q1)[:, s], oq) <= TOL[dtype], b
        assert rel_err(host(p1)[:, s], op) <= TOL[dtype], b


def test_graph_replays_match_direct_launches():
    """Shoots whose steps replay a captured hipGraph (several graph sizes, with a remainder
    launched directly, and eager work on the stream between calls) give bitwise the result
    of launching every kernel directly."""
    offs, q, p = ragged_batch([40, 300, 129, 7], 2, seed=303, pscale=0.3)
    prm = lm.make_params(2, lm.CONON, 0.2)
    t = lm.lm_batch_default_tuning(offs)
    out = {}
    for gs in [0, 1, 3, 7, 3]:
        t.graph_steps = gs
        q1, p1 = torch.empty_like(dev(q)), torch.empty_like(dev(q))
        lm.lm_shoot_batched(prm, offs, dev(q), dev(p), 0.9, 7, q1, p1, tuning=t)
        # eager work between the replays
        dq, dp = torch.empty_like(q1), torch.empty_like(q1)
        lm.lm_rhs_batched(prm, offs, q1, p1, dq, dp)
        torch.cuda.synchronize()
        out.setdefault(gs, []).append((host(q1), host(p1)))
    ref_q, ref_p = out[0][0]
    for gs, runs in out.items():
        for gq, gp in runs:
            assert np.array_equal(gq, ref_q) and np.array_equal(gp, ref_p), gs
    for b in range(4):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.shoot(q[:, s], p[:, s], lm.CONON, 0.2, 7, T=0.9)
        assert rel_err(ref_q[:, s], oq) <= 1e-10 and rel_err(ref_p[:, s], op) <= 1e-10


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_autotune_picks_a_valid_shape(dtype):
    sizes, offs, X, Y = curve_batch(12, 2000)
    Xd = dev(rounded(X, dtype), dtype)
    pd = dev(rounded(0.05 * (Y - X), dtype), dtype)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=dtype)
    t = lm.lm_batch_autotune(prm, offs, Xd, pd)
    print("tuned:", t.as_dict())
    assert t.stage_us > 0.0
    assert t.groups >= 0 and t.graph_steps >= 0 and all(1 <= s <= 64 for s in t.split)
    assert t.bucket_max[len(t.bucket_max) - 1] >= int(sizes.max())
    # the tuned shape computes the same shoot as the default one
    a = [torch.empty_like(Xd) for _ in range(4)]
    lm.lm_shoot_batched(prm, offs, Xd, pd, 1.0, 5, a[0], a[1], tuning=t)
    lm.lm_shoot_batched(prm, offs, Xd, pd, 1.0, 5, a[2], a[3])
    torch.cuda.synchronize()
    assert rel_err(host(a[0]), host(a[2])) <= TOL[dtype] * 0.1
    assert rel_err(host(a[1]), host(a[3])) <= TOL[dtype] * 0.1


# LM_BATCH_FILL: waves per SIMD below which a match's shoots split their one-sided problems'
# sources further (unset: the library's default; "0": the tuning's splits only; "8": splits up to
# one chunk per source point on these small problems)
FILLS = [None, "0", "8"]


def set_fill(monkeypatch, fill):
    if fill is None:
        monkeypatch.delenv("LM_BATCH_FILL", raising=False)
    else:
        monkeypatch.setenv("LM_BATCH_FILL", fill)


@pytest.mark.parametrize("fill", FILLS)
def test_batched_feedback_matches_oracle_per_problem(fill, monkeypatch):
    set_fill(monkeypatch, fill)
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=20,
                                                    max_iter=200, q1=q1)
    assert st == lm.LM_OK and all(s == lm.LM_OK for s in stats)
    gp, gq = host(p0), host(q1)
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-6, 20, max_iter=200)
        assert ref.status == 0
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert infos[b].shoots == infos[b].iters     # from rest: the first shoot is the identity map
        assert abs(infos[b].resid_inf - ref.resid) <= 1e-9
        assert rel_err(gp[:, s], ref.p0) <= 1e-8
        assert rel_err(gq[:, s], ref.q1) <= 1e-10
        assert abs(infos[b].H - ref.H) <= 1e-9 * abs(ref.H)


def test_batched_inexact_feedback_matches_oracle_per_problem():
    """The inexact system (tau > 0: the tau p_i advection term and the (K + tau I) update,
    equation "N-particle-inexact") through batched Algorithm 1: per problem the oracle's
    iteration count, momenta, q(1), and H of equation "H" (the kernel form alone, without tau)."""
    tau = 0.05
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1, tau=tau)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=20,
                                                    max_iter=200, q1=q1)
    assert st == lm.LM_OK and all(s == lm.LM_OK for s in stats)
    gp, gq = host(p0), host(q1)
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-6, 20, max_iter=200, tau=tau)
        assert ref.status == 0
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert rel_err(gp[:, s], ref.p0) <= 1e-8
        assert rel_err(gq[:, s], ref.q1) <= 1e-10
        assert abs(infos[b].H - ref.H) <= 1e-9 * abs(ref.H)
        assert abs(infos[b].H - oracle.hamiltonian(X[:, s], ref.p0, lm.CONON, 0.1)) <= 1e-9 * abs(ref.H)


@pytest.mark.parametrize("fill", FILLS)
def test_batched_feedback_single_precision_shoots(fill, monkeypatch):
    set_fill(monkeypatch, fill)
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=lm.F32)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-5, steps=20,
                                                    max_iter=200)
    assert st == lm.LM_OK
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-5, 20, max_iter=200)
        assert abs(infos[b].iters - ref.iters) <= 1, (b, infos[b].iters, ref.iters)
        assert infos[b].resid_inf < 1e-5
        assert rel_err(host(p0)[:, s], ref.p0) <= 1e-3


def test_batched_feedback_switches_to_double_precision():
    """Single-precision shoots until a problem's residual is below f32_switch, then double:
    every problem reaches a tolerance below what single-precision shoots can resolve, with
    the oracle's iteration count (one more update at most: the last single-precision
    direction is slightly off)."""
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=lm.F32)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-9, steps=20,
                                                    max_iter=200, q1=q1, f32_switch=1e-4)
    assert st == lm.LM_OK, stats
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-9, 20, max_iter=200)
        assert ref.status == 0
        assert 0 <= infos[b].iters - ref.iters <= 1, (b, infos[b].iters, ref.iters)
        assert infos[b].resid_inf < 1e-9
        # the reported q(1) is a double-precision shoot of the returned momenta
        oq, _ = oracle.shoot(X[:, s], host(p0)[:, s], lm.CONON, 0.1, 20)
        assert rel_err(host(q1)[:, s], oq) <= 1e-10
        assert np.max(np.abs(oq - Y[:, s])) < 1e-9


def test_batched_feedback_single_precision_floor_switches_to_double():
    """f32_switch below the single-precision floor (1e-12): each problem's residual stops
    falling at its floor, where the problem switches to double precision; every problem
    reaches tol = 1e-9 within two updates of the oracle's count (either way: the single-precision
    updates before the switch move its residuals slightly)."""
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=lm.F32)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-9, steps=20,
                                                    max_iter=200, f32_switch=1e-12)
    assert st == lm.LM_OK, stats
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-9, 20, max_iter=200)
        assert ref.status == 0
        assert infos[b].resid_inf < 1e-9
        assert abs(infos[b].iters - ref.iters) <= 2, (b, infos[b].iters, ref.iters)


@pytest.mark.parametrize("wide_min", [None, "0", "4096"])
def test_batched_feedback_multi_panel_problems_in_the_batched_solve(wide_min, monkeypatch):
    """Problems of 40, 1000 and 2900 points (1, 8 and 23 diagonal blocks, ragged last blocks)
    through both batched solves: LM_BATCH_WIDE_MIN = 4096 puts all three in the one-workgroup
    kernel (its sweeps take their unrolled and remainder loops at every block), 0 all three in
    the wide sweeps (many workgroups per problem), the default (1024) the largest in the wide
    sweeps beside the others in the one-workgroup kernel; iteration counts and momenta are the
    oracle's."""
    if wide_min is None:
        monkeypatch.delenv("LM_BATCH_WIDE_MIN", raising=False)
    else:
        monkeypatch.setenv("LM_BATCH_WIDE_MIN", wide_min)
    sizes = [40, 1000, 2900]
    parts = [inputs.config_curve2d(n, seed=[321, n]) for n in sizes]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.concatenate([pr.X for pr in parts], axis=1)
    Y = np.concatenate([pr.Y for pr in parts], axis=1)
    prm = lm.make_params(2, lm.CONON, 0.1)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=10,
                                                    max_iter=100)
    assert st == lm.LM_OK
    for b in range(3):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-6, 10, max_iter=100)
        assert ref.status == 0
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert rel_err(host(p0)[:, s], ref.p0) <= 1e-8


def test_batched_feedback_wide_solves_in_three_dimensions(monkeypatch):
    """The wide sweeps with three components: two sphere problems of 300 and 1500 points
    (3 and 12 blocks), every problem in the wide sweeps; iteration counts and momenta are the
    oracle's."""
    monkeypatch.setenv("LM_BATCH_WIDE_MIN", "0")
    sizes = [300, 1500]
    parts = [inputs.config_sphere3d(n, seed=[322, n], sigma=0.15) for n in sizes]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.concatenate([pr.X for pr in parts], axis=1)
    Y = np.concatenate([pr.Y for pr in parts], axis=1)
    prm = lm.make_params(3, lm.CONON, 0.15)
    p0 = torch.zeros((3, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=10,
                                                    max_iter=100)
    assert st == lm.LM_OK, stats
    for b in range(2):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.15, 0.8, 1e-6, 10, max_iter=100)
        assert ref.status == 0
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert rel_err(host(p0)[:, s], ref.p0) <= 1e-8


def test_batched_feedback_with_a_problem_too_large_for_the_batched_solve():
    """A problem above the one-workgroup solve's limit (4096 points) is solved by the wide
    sweeps in place in the concatenated layout; its iteration count and momenta are the
    oracle's, as are those of the small problem beside it."""
    sizes = [40, 4100]
    parts = [inputs.config_curve2d(n, seed=[320, n]) for n in sizes]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.concatenate([pr.X for pr in parts], axis=1)
    Y = np.concatenate([pr.Y for pr in parts], axis=1)
    prm = lm.make_params(2, lm.CONON, 0.1)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=10,
                                                    max_iter=100)
    assert st == lm.LM_OK
    for b in range(2):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-6, 10, max_iter=100)
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert rel_err(host(p0)[:, s], ref.p0) <= 1e-8


def test_batched_feedback_reports_each_problems_outcome():
    """A problem whose K is singular (every landmark at one point: K is the all-ones matrix)
    stops at once with LM_ESINGULAR while the others converge; with too few iterations
    every problem ends LM_ENOTCONV."""
    sizes, offs, X, Y = curve_batch(4, 200)
    X0 = X
    X = X.copy()
    s1 = slice(offs[1], offs[2])
    X[:, s1] = X[:, offs[1]][:, None]
    prm = lm.make_params(2, lm.CONON, 0.1)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=20,
                                                    max_iter=200)
    assert st == lm.LM_ESINGULAR
    assert stats[1] == lm.LM_ESINGULAR and infos[1].iters == 0
    assert np.all(host(p0)[:, s1] == 0.0)
    for b in (0, 2, 3):
        assert stats[b] == lm.LM_OK
    p0.zero_()
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X0), dev(Y), p0, h=0.8, tol=1e-6, steps=20,
                                                    max_iter=3)
    assert st == lm.LM_ENOTCONV and all(s == lm.LM_ENOTCONV for s in stats)
    assert all(i.iters == 3 for i in infos)


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_full_batch_sampled_rhs(dtype):
    """The 256-problem workload (sizes log-uniform in [32, 4096]) with the autotuned shape:
    the smallest, a middle and the largest problem against the oracle."""
    sizes, offs, X, Y = inputs.config_batched()
    q = rounded(X, dtype)
    p = rounded(np.concatenate([inputs.bench_momentum(X[:, offs[b]:offs[b + 1]], Y[:, offs[b]:offs[b + 1]],
                                                      inputs.curve_kernel_mass(int(sizes[b]), 2 * np.pi, 0.1, 0))
                                for b in range(len(sizes))], axis=1), dtype)
    prm = lm.make_params(2, lm.CONON, 0.1, dtype=dtype)
    qd, pd = dev(q, dtype), dev(p, dtype)
    t = lm.lm_batch_autotune(prm, offs, qd, pd)
    dq, dp = torch.empty_like(qd), torch.empty_like(qd)
    lm.lm_rhs_batched(prm, offs, qd, pd, dq, dp, tuning=t)
    torch.cuda.synchronize()
    order = np.argsort(sizes)
    for b in [int(order[0]), int(order[len(order) // 2]), int(order[-1])]:
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.rhs(q[:, s], p[:, s], lm.CONON, 0.1)
        assert rel_err(host(dq)[:, s], oq) <= TOL[dtype], (b, sizes[b])
        assert rel_err(host(dp)[:, s], op) <= TOL[dtype], (b, sizes[b])


# ------------------------------------------------------------------ symmetric problems


def _sym_tuning(offs, sym_min, waves, split=1):
    t = lm.lm_batch_default_tuning(offs)
    t.sym_min = sym_min
    t.sym_waves = waves
    for k in range(len(t.split)):
        t.split[k] = split
    return t


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("dim,kernel,tau", [(2, lm.CONON, 0.0), (3, lm.CONON, 0.1), (2, lm.GAUSS, 0.2),
                                            (3, lm.GAUSS, 0.0)])
def test_batched_symmetric_rhs_matches_oracle(dim, kernel, tau, waves, dtype):
    """Every problem symmetric (sym_min = 1), at every width: ragged tiles and superblocks,
    one-point and one-tile problems."""
    offs, q, p = ragged_batch(SIZES + [1100], dim, seed=304)
    q, p = rounded(q, dtype), rounded(p, dtype)
    prm = lm.make_params(dim, kernel, 0.3, tau=tau, dtype=dtype)
    dq, dp = torch.empty_like(dev(q, dtype)), torch.empty_like(dev(q, dtype))
    lm.lm_rhs_batched(prm, offs, dev(q, dtype), dev(p, dtype), dq, dp, tuning=_sym_tuning(offs, 1, waves))
    torch.cuda.synchronize()
    gq, gp = host(dq), host(dp)
    for b in range(len(offs) - 1):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.rhs(q[:, s], p[:, s], kernel, 0.3, tau)
        assert rel_err(gq[:, s], oq) <= TOL[dtype], (b, rel_err(gq[:, s], oq))
        if offs[b + 1] - offs[b] > 1:
            assert rel_err(gp[:, s], op) <= TOL[dtype], (b, rel_err(gp[:, s], op))
        else:
            assert np.all(gp[:, s] == 0.0)


def test_batched_mixed_symmetric_and_split_problems():
    """Problems from 200 points symmetric, the smaller ones one-sided with split sums, in the
    same stage, in both precisions."""
    offs, q, p = ragged_batch(SIZES + [1100], 2, seed=305)
    for dtype in (lm.F64, lm.F32):
        qq, pp = rounded(q, dtype), rounded(p, dtype)
        prm = lm.make_params(2, lm.CONON, 0.25, dtype=dtype)
        dq, dp = torch.empty_like(dev(qq, dtype)), torch.empty_like(dev(qq, dtype))
        lm.lm_rhs_batched(prm, offs, dev(qq, dtype), dev(pp, dtype), dq, dp, tuning=_sym_tuning(offs, 200, 2, 4))
        torch.cuda.synchronize()
        for b in range(len(offs) - 1):
            s = slice(offs[b], offs[b + 1])
            oq, op = oracle.rhs(qq[:, s], pp[:, s], lm.CONON, 0.25)
            assert rel_err(host(dq)[:, s], oq) <= TOL[dtype], (dtype, b)
            if offs[b + 1] - offs[b] > 1:
                assert rel_err(host(dp)[:, s], op) <= TOL[dtype], (dtype, b)


@pytest.mark.parametrize("dtype", [lm.F64, lm.F32])
def test_batched_symmetric_shoot_graph_replays_and_oracle(dtype):
    """Problems from 100 points symmetric, graph-replayed and direct.  Single precision runs
    curves like the matching workloads: on the random states the shoot amplifies rounding so
    much that the FP32 one-sided kernel itself lands 5e-4 from the oracle in p (FP64 8e-12)."""
    if dtype == lm.F64:
        offs, q, p = ragged_batch([40, 300, 1029, 7, 513], 2, seed=306, pscale=0.3)
        sigma, T, steps = 0.2, 0.9, 7
    else:
        sizes, offs, q, Y = curve_batch(6, 1100)
        p = np.concatenate([inputs.bench_momentum(q[:, offs[b]:offs[b + 1]], Y[:, offs[b]:offs[b + 1]],
                                                  inputs.curve_kernel_mass(int(sizes[b]), 2 * np.pi, 0.1, 0))
                            for b in range(len(sizes))], axis=1)
        sigma, T, steps = 0.1, 1.0, 20
        assert max(sizes) >= 100
    q, p = rounded(q, dtype), rounded(p, dtype)
    prm = lm.make_params(2, lm.CONON, sigma, dtype=dtype)
    t = _sym_tuning(offs, 100, 2)
    out = []
    for gs in [0, 3, 0]:
        t.graph_steps = gs
        q1, p1 = torch.empty_like(dev(q, dtype)), torch.empty_like(dev(q, dtype))
        lm.lm_shoot_batched(prm, offs, dev(q, dtype), dev(p, dtype), T, steps, q1, p1, tuning=t)
        torch.cuda.synchronize()
        out.append((host(q1), host(p1)))
    for gq, gp in out[1:]:
        assert np.array_equal(gq, out[0][0]) and np.array_equal(gp, out[0][1])
    for b in range(len(offs) - 1):
        s = slice(offs[b], offs[b + 1])
        oq, op = oracle.shoot(q[:, s], p[:, s], lm.CONON, sigma, steps, T=T)
        assert rel_err(out[0][0][:, s], oq) <= TOL[dtype] and rel_err(out[0][1][:, s], op) <= TOL[dtype], b


def test_batched_symmetric_feedback_matches_oracle_per_problem():
    sizes, offs, X, Y = curve_batch(5, 300)
    prm = lm.make_params(2, lm.CONON, 0.1)
    p0 = torch.zeros((2, int(offs[-1])), dtype=torch.float64, device=DEV)
    q1 = torch.empty_like(p0)
    st, infos, stats = lm.lm_feedback_match_batched(prm, offs, dev(X), dev(Y), p0, h=0.8, tol=1e-6, steps=20,
                                                    max_iter=200, q1=q1, tuning=_sym_tuning(offs, 1, 1))
    assert st == lm.LM_OK and all(s == lm.LM_OK for s in stats)
    gp, gq = host(p0), host(q1)
    for b in range(len(sizes)):
        s = slice(offs[b], offs[b + 1])
        ref = oracle.feedback_match(X[:, s], Y[:, s], lm.CONON, 0.1, 0.8, 1e-6, 20, max_iter=200)
        assert infos[b].iters == ref.iters, (b, infos[b].iters, ref.iters)
        assert rel_err(gp[:, s], ref.p0) <= 1e-8
        assert rel_err(gq[:, s], ref.q1) <= 1e-10
