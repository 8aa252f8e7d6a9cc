"""Host-side logic of the batched entry points (no GPU needed): the default launch shape,
and the argument checks that run before any HIP call."""

import ctypes

import numpy as np
import pytest

import inputs
from paper_1510_03816_amd import _lib


def test_default_tuning_covers_the_256_problem_workload():
    sizes, offs, X, Y = inputs.config_batched()
    assert len(sizes) == 256 and offs[0] == 0 and offs[-1] == sizes.sum()
    assert 32 <= sizes.min() and sizes.max() <= 4096
    t = _lib.lm_batch_default_tuning(offs)
    bm = list(t.bucket_max)
    assert bm == sorted(bm) and bm[-1] >= sizes.max()
    assert all(s == 1 for s in t.split) and t.groups >= 0 and t.graph_steps >= 0
    assert t.sym_min > 0 and t.sym_waves in (1, 2, 4, 8)


@pytest.mark.parametrize("offs", [[], [1, 5], [0, 0, 3], [0, 4, 3], [0, 5, 5]])
def test_bad_offsets_rejected(offs):
    if len(offs) == 0:
        t = _lib.lm_batch_tuning()
        rc = _lib.load().lm_batch_default_tuning(0, (ctypes.c_int64 * 1)(0), ctypes.byref(t))
        assert rc == _lib.LM_EINVAL
        return
    with pytest.raises(_lib.LmError) as e:
        _lib.lm_batch_default_tuning(offs)
    assert e.value.status == _lib.LM_EINVAL


def _rhs_batched_rc(offs, tuning=None, **kw):
    prm = _lib.make_params(2, _lib.CONON, 0.5, **kw)
    B, arr = _lib._offs_array(offs)
    a, b, c, d = (ctypes.c_void_p(v) for v in (16, 32, 48, 64))
    return _lib.load().lm_rhs_batched(ctypes.byref(prm), B, arr, a, b, c, d,
                                      None if tuning is None else ctypes.byref(tuning), None)


def test_bad_tuning_rejected_before_any_launch():
    offs = [0, 10, 300]
    t = _lib.lm_batch_default_tuning(offs)
    t.split[0] = 0
    assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL
    t = _lib.lm_batch_default_tuning(offs)
    t.bucket_max[3] = 100                      # below the largest problem (290)
    assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL
    t = _lib.lm_batch_default_tuning(offs)
    t.bucket_max[1] = 5                        # not ascending
    assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL
    t = _lib.lm_batch_default_tuning(offs)
    t.groups = -1
    assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL
    t = _lib.lm_batch_default_tuning(offs)
    t.sym_min = -1
    assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL
    for bad in (0, 3, 16):
        t = _lib.lm_batch_default_tuning(offs)
        t.sym_waves = bad
        assert _rhs_batched_rc(offs, t) == _lib.LM_EINVAL


def test_cutoff_and_inexact_stop_rule_unsupported_for_batches():
    assert _rhs_batched_rc([0, 10, 20], cutoff=0.5) == _lib.LM_EUNSUPPORTED
    prm = _lib.make_params(2, _lib.CONON, 0.5)
    o = _lib.lm_match_opts(0.8, 1e-6, 10, 10, 1, 0, 0.0, None, 0, 0)
    B, arr = _lib._offs_array([0, 10, 20])
    infos = (_lib.lm_match_info * B)()
    stats = (ctypes.c_int32 * B)()
    p = ctypes.c_void_p(16)
    rc = _lib.load().lm_feedback_match_batched(ctypes.byref(prm), ctypes.byref(o), B, arr, p, p, p, None, infos,
                                               stats, None, None)
    assert rc == _lib.LM_EUNSUPPORTED


def test_aliased_outputs_rejected():
    prm = _lib.make_params(2, _lib.CONON, 0.5)
    B, arr = _lib._offs_array([0, 10])
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    rc = _lib.load().lm_rhs_batched(ctypes.byref(prm), B, arr, a, b, a, ctypes.c_void_p(64), None, None)
    assert rc == _lib.LM_EINVAL
