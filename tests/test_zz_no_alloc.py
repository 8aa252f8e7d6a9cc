"""lm_shoot_noalloc, the shoot that allocates nothing (its scratch is the library's fixed
per-GPU array), against lm_shoot on the same inputs, through the C ABI (needs an MI355X).

Two calls in a row share the array, the second with a smaller input: the second must not see
anything the first left behind.  Results must equal lm_shoot's (same kernels, same order:
bitwise), which the parity tests tie to the oracle; one case is also checked against the
oracle directly.
"""

import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_1510_03816_amd as lm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {lm.F64: torch.float64, lm.F32: torch.float32}
TOL = {lm.F64: 1e-10, lm.F32: 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)


def rel_err(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def problem(n, dim):
    pr = inputs.config_sphere3d(n, sigma=0.1) if dim == 3 else inputs.config_curve2d(n, sigma=0.1)
    return pr.X, pr.p_bench()


def both(prm, q0, p0, t1, steps):
    """(lm_shoot result, lm_shoot_noalloc result) as host arrays."""
    dt = TDT[prm.dtype]
    q = torch.tensor(q0, dtype=dt, device=DEV)
    p = torch.tensor(p0, dtype=dt, device=DEV)
    qa, pa, qb, pb = (torch.empty_like(q) for _ in range(4))
    lm.lm_shoot(prm, q, p, t1, steps, qa, pa)
    lm.lm_shoot_noalloc(prm, q, p, t1, steps, qb, pb)
    torch.cuda.synchronize()
    return [t.double().cpu().numpy() for t in (qa, pa, qb, pb)]


# each sequence runs in order on the one shared array, the later calls smaller
SEQUENCES = {
    "f64_3d": [(lm.F64, 3, lm.CONON, 9000, 3), (lm.F64, 3, lm.CONON, 3001, 4), (lm.F64, 2, lm.GAUSS, 200, 6)],
    "f32_mixed": [(lm.F32, 3, lm.GAUSS, 6000, 3), (lm.F32, 2, lm.CONON, 777, 5)],
}


@pytest.mark.parametrize("name", sorted(SEQUENCES))
def test_noalloc_shoot_equals_lm_shoot_on_consecutive_calls(name):
    for dtype, dim, kernel, n, steps in SEQUENCES[name]:
        q0, p0 = problem(n, dim)
        prm = lm.make_params(dim, kernel, 0.1, dtype=dtype)
        qa, pa, qb, pb = both(prm, q0, p0, 0.05 * steps, steps)
        eq, ep = rel_err(qb, qa), rel_err(pb, pa)
        same = np.array_equal(qa, qb) and np.array_equal(pa, pb)
        print("%s n=%d dim=%d dtype=%d: rel diff q %.2e p %.2e, bitwise %s, plan %s" % (
            name, n, dim, dtype, eq, ep, same, lm.lm_pair_plan(prm, n)))
        assert eq <= TOL[dtype] and ep <= TOL[dtype]
        assert same


def test_noalloc_shoot_matches_oracle_and_runs_in_place():
    q0, p0 = problem(3001, 3)
    prm = lm.make_params(3, lm.CONON, 0.1)
    q = torch.tensor(q0, device=DEV)
    p = torch.tensor(p0, device=DEV)
    lm.lm_shoot_noalloc(prm, q, p, 0.1, 2, q, p)          # in place
    torch.cuda.synchronize()
    oq, op = oracle.shoot(q0, p0, lm.CONON, 0.1, 2, T=0.1)
    assert rel_err(q.cpu().numpy(), oq) <= 1e-10 and rel_err(p.cpu().numpy(), op) <= 1e-10


def test_noalloc_shoot_refuses_what_it_cannot_hold():
    q0, p0 = problem(24576, 3)                 # its partial sums alone exceed the array
    prm = lm.make_params(3, lm.CONON, 0.05)
    q = torch.tensor(q0, device=DEV)
    p = torch.tensor(p0, device=DEV)
    q1, p1 = torch.empty_like(q), torch.empty_like(p)
    with pytest.raises(lm.LmError) as e:
        lm.lm_shoot_noalloc(prm, q, p, 1.0, 1, q1, p1)
    assert e.value.status == lm.LM_ENOMEM and "bytes of scratch" in str(e.value)
    with pytest.raises(lm.LmError) as e:
        lm.lm_shoot_noalloc(lm.make_params(3, lm.CONON, 0.05, cutoff=0.3), q, p, 1.0, 1, q1, p1)
    assert e.value.status == lm.LM_EUNSUPPORTED
    # the refused calls left the array usable: the largest documented size, then a small one
    for n in (16384, 2000):
        q0, p0 = problem(n, 3)
        qa, pa, qb, pb = both(lm.make_params(3, lm.CONON, 0.1), q0, p0, 0.02, 1)
        assert np.array_equal(qa, qb) and np.array_equal(pa, pb)
