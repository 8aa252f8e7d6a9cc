"""The pair-sum launch plan (host logic, no GPU): which kernel a size and precision get, the
symmetric kernel's superblock arithmetic, and the environment overrides."""

import os

import pytest

import paper_1510_03816_amd as lm


@pytest.fixture(autouse=True)
def _clean_env(monkeypatch):
    monkeypatch.delenv("LM_SYM", raising=False)
    monkeypatch.delenv("LM_SYM_WAVES", raising=False)
    monkeypatch.delenv("LM_SYM_ROWS", raising=False)
    monkeypatch.delenv("LM_SMALL", raising=False)
    monkeypatch.delenv("LM_SMALL_WAVES", raising=False)


def plan(n, dtype=lm.F64, cutoff=0.0, dim=3):
    prm = lm.make_params(dim, lm.CONON, 0.05, dtype=dtype, cutoff=cutoff)
    return lm.lm_pair_plan(prm, n)


def sym(T, w, rows=2):
    """Superblock count, workgroups and partial slots of the symmetric kernel for T tiles."""
    S = -(-T // (rows * w))
    return S, S * (S + 1) // 2, S + 1


def test_full_size_double_uses_the_wide_symmetric_tier():
    """Four row tiles per wave, two waves per workgroup: superblocks of 8 tiles."""
    S, wg, slots = sym(1024, 2, 4)
    assert plan(65536) == {"symmetric": 1, "waves": 2, "workgroups": wg, "partial_slots": slots, "small": 0,
                           "rows": 4}
    assert (S, wg, slots) == (128, 8256, 129)


@pytest.mark.parametrize("n,waves,rows", [(8129, 1, 2), (8192, 1, 2), (12224, 1, 2), (12288, 2, 2), (16384, 2, 2),
                                          (49088, 2, 2), (49089, 2, 4), (131072, 2, 4)])
def test_size_rule(n, waves, rows):
    p = plan(n)
    T = -(-n // 64)
    assert p["symmetric"] == 1 and p["waves"] == waves and p["rows"] == rows
    assert (p["workgroups"], p["partial_slots"]) == sym(T, waves, rows)[1:]


@pytest.mark.parametrize("n", [1, 257, 4096, 8128])
def test_small_sizes_keep_one_sided_kernel(n):
    p = plan(n)
    assert p["symmetric"] == 0 and p["waves"] == 4 and p["rows"] == 1
    assert p["small"] == (1 if n <= 128 else 0)


@pytest.mark.parametrize("n,dim,dtype,small", [
    (1, 2, lm.F64, 1), (128, 2, lm.F64, 1), (129, 2, lm.F64, 0), (128, 3, lm.F32, 1), (129, 3, lm.F32, 0),
    (256, 2, lm.F32, 0),
])
def test_one_workgroup_shoot_sizes(n, dim, dtype, small, monkeypatch):
    """Shoots run whole inside one workgroup up to 128 points, where that beats one launch per
    stage; never with tile skipping.  LM_SMALL forces either path (1: up to 256 points)."""
    assert lm.lm_pair_plan(lm.make_params(dim, lm.CONON, 0.3, dtype=dtype), n)["small"] == small
    assert lm.lm_pair_plan(lm.make_params(dim, lm.CONON, 0.3, dtype=dtype, cutoff=0.5), n)["small"] == 0
    monkeypatch.setenv("LM_SMALL", "1")
    assert lm.lm_pair_plan(lm.make_params(dim, lm.CONON, 0.3, dtype=dtype), n)["small"] == (1 if n <= 256 else 0)
    monkeypatch.setenv("LM_SMALL", "0")
    assert lm.lm_pair_plan(lm.make_params(dim, lm.CONON, 0.3, dtype=dtype), n)["small"] == 0


def test_one_sided_split_rule(monkeypatch):
    # 128 target tiles: 16384 workgroups wanted, capped at 16 source splits from 128 tiles on
    monkeypatch.setenv("LM_SYM", "0")
    p = plan(8192)
    assert p == {"symmetric": 0, "waves": 4, "workgroups": 128 * 16, "partial_slots": 16, "small": 0, "rows": 1}
    monkeypatch.delenv("LM_SYM")
    # 64 tiles of 2-D points: 256 splits wanted, limited to 64 (and by the 32-source chunk floor)
    p = plan(4096, dim=2)
    assert p["workgroups"] == 64 * 32 and p["partial_slots"] == 32
    # 94 tiles: 16 splits from 80 tiles on
    p = plan(6000)
    assert p["symmetric"] == 0 and p["workgroups"] == 94 * 16 and p["partial_slots"] == 16
    p = plan(5056)          # 79 tiles: 39 splits (the 32-source chunk floor)
    assert p["workgroups"] == 79 * 39 and p["partial_slots"] == 39


@pytest.mark.parametrize("n,waves", [(16320, 0), (16321, 1), (24576, 1), (32704, 1), (32705, 2), (49088, 2),
                                     (49089, 4), (65536, 4), (131072, 4)])
def test_single_precision_size_rule(n, waves):
    """Single precision: the one-sided kernel below 256 tiles, then the symmetric kernel with
    two row tiles per wave: one wave, two from 512 tiles, four from 768."""
    p = plan(n, dtype=lm.F32)
    T = -(-n // 64)
    if waves == 0:
        assert p["symmetric"] == 0
    else:
        assert p["symmetric"] == 1 and p["waves"] == waves and p["rows"] == 2
        assert (p["workgroups"], p["partial_slots"]) == sym(T, waves)[1:]


def test_cutoff_size_rule():
    p = plan(65536, cutoff=0.3)                 # tile skipping: two rows, two waves, 4-tile superblocks
    assert p["symmetric"] == 1 and p["rows"] == 2 and p["waves"] == 2 and p["partial_slots"] == 257
    assert plan(49088, cutoff=0.3)["symmetric"] == 0        # 768 tiles needed with tile skipping
    assert plan(49152, cutoff=0.3)["symmetric"] == 1
    p = plan(65536, dtype=lm.F32, cutoff=0.3)   # single precision: the same shape
    assert p["symmetric"] == 1 and p["rows"] == 2 and p["waves"] == 2 and p["partial_slots"] == 257
    assert plan(49088, dtype=lm.F32, cutoff=0.3)["symmetric"] == 0
    assert plan(100, cutoff=0.3)["small"] == 0


def test_environment_overrides(monkeypatch):
    monkeypatch.setenv("LM_SYM", "0")
    assert plan(65536)["symmetric"] == 0
    monkeypatch.setenv("LM_SYM", "1")
    p = plan(1000)                       # 16 tiles, one wave per workgroup
    assert p["symmetric"] == 1 and p["waves"] == 1 and p["partial_slots"] == 9 and p["workgroups"] == 36
    monkeypatch.setenv("LM_SYM_WAVES", "8")
    p = plan(65536)
    assert p["waves"] == 8 and p["rows"] == 2 and (p["workgroups"], p["partial_slots"]) == sym(1024, 8)[1:]
    monkeypatch.setenv("LM_SYM_ROWS", "4")
    assert plan(65536)["rows"] == 2                   # four rows take at most four waves
    monkeypatch.setenv("LM_SYM_WAVES", "4")
    p = plan(65536)
    assert p["waves"] == 4 and p["rows"] == 4 and (p["workgroups"], p["partial_slots"]) == sym(1024, 4, 4)[1:]
    assert plan(65536, dtype=lm.F32)["rows"] == 4     # forced: four rows in single precision too
    monkeypatch.delenv("LM_SYM_ROWS")
    monkeypatch.setenv("LM_SYM_WAVES", "3")   # not a width: the size rule applies
    assert plan(65536)["waves"] == 2 and plan(65536)["rows"] == 4
    monkeypatch.delenv("LM_SYM_WAVES")
    monkeypatch.setenv("LM_SYM_ROWS", "2")    # two rows in the wide tier: four waves
    assert plan(65536)["waves"] == 4 and plan(65536)["rows"] == 2


def test_invalid_arguments():
    with pytest.raises(lm.LmError):
        plan(0)


def test_device_exponential_constants_are_the_generators():
    """The hex constants of the device exponentials in lm_math.h (degree 9 for the pair sums,
    degree 10 for the dense kernel matrix) are exactly what gen_exp_coeffs.py derives, and the
    polynomials they form stay within 4e-14 and 6e-16 of 2^f on the reduced interval
    (evaluated in high precision from the rounded coefficients)."""
    import re
    import subprocess
    import sys
    import mpmath as mp
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1510_03816_amd", "csrc")
    src = open(os.path.join(csrc, "lm_math.h")).read()
    mp.mp.dps = 40
    for fn, deg, bound in [("exp2_nonpos(", 9, 4e-14), ("exp2_nonpos_fine(", 10, 6e-16)]:
        out = subprocess.run([sys.executable, os.path.join(csrc, "gen_exp_coeffs.py"), str(deg)],
                             stdout=subprocess.PIPE, text=True, check=True).stdout
        want = [float.fromhex(v) for v in re.findall(r"^C\d+\s*=\s*(\S+)$", out, flags=re.M)]
        start = src.index("double " + fn)
        body = src[src.index("double p = ", start):src.index("return __builtin_ldexp", start)]
        got = [float.fromhex(v) if v.startswith("0x") else float(v)
               for v in re.findall(r"(0x1\.[0-9a-f]+p-?\d+|1\.0)\)?;", body)]
        assert got == want and len(got) == deg + 1, fn
        worst = 0
        for t in mp.linspace(-0.5, 0.5, 801):
            pv = mp.mpf(0)
            for c in got:
                pv = pv * t + mp.mpf(c)
            worst = max(worst, abs(pv / mp.power(2, t) - 1))
        assert worst < bound, fn
