"""The C ABI library loads and exports every symbol include/liblm.h declares (no GPU needed).

Argument validation happens before any HIP call, so the invalid-argument statuses can be
checked on a machine without a GPU as well.
"""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "liblm.h")
LIB = os.path.join(ROOT, "paper_1510_03816_amd", "liblm.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblm.so is not built: run python __graft_entry__.py (build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_paths_entry_points():
    names = header_functions()
    for want in ["lm_rhs", "lm_shoot", "lm_feedback_match", "lm_hamiltonian", "lm_ksolve",
                 "lm_velocity", "lm_last_error"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r"\bT (lm_\w+)", out))
    for name in header_functions():
        assert name in exported, name
        getattr(lib, name)


def test_binding_lists_every_declared_symbol():
    from paper_1510_03816_amd import _lib
    assert sorted(_lib.EXPORTS) == header_functions()


def test_package_exposes_every_binding():
    import paper_1510_03816_amd as pkg
    from paper_1510_03816_amd import _lib
    for name in _lib.EXPORTS:
        if name != "lm_last_error":            # exposed as last_error()
            assert callable(getattr(pkg, name)), name


def test_struct_layouts_match_header(tmp_path):
    """Compile a C probe against the header and compare every field offset with ctypes."""
    from paper_1510_03816_amd import _lib
    structs = {"lm_params": _lib.lm_params, "lm_match_opts": _lib.lm_match_opts,
               "lm_match_info": _lib.lm_match_info, "lm_step_info": _lib.lm_step_info,
               "lm_lbfgs_opts": _lib.lm_lbfgs_opts, "lm_lbfgs_info": _lib.lm_lbfgs_info,
               "lm_batch_tuning": _lib.lm_batch_tuning, "lm_plan_info": _lib.lm_plan_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "liblm.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (sname, sname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sname, fname, sname, fname))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for sname, cls in structs.items():
        assert int(got[sname]) == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(got[sname + "." + fname]) == getattr(cls, fname).offset, (sname, fname)


def _params(dim=2, kernel=0, dtype=0, sigma=0.5, tau=0.0, cutoff=0.0, flags=0):
    from paper_1510_03816_amd import _lib
    return _lib.lm_params(dim, kernel, dtype, flags, sigma, tau, cutoff)


@pytest.mark.parametrize("kw,status", [
    (dict(dim=4), -1), (dict(kernel=7), -1), (dict(dtype=3), -1), (dict(sigma=0.0), -1),
    (dict(sigma=float("nan")), -1), (dict(tau=-1.0), -1), (dict(flags=1), -1),
    (dict(cutoff=-1.0), -1),
])
def test_invalid_params_rejected_before_any_launch(lib, kw, status):
    p = _params(**kw)
    dummy = ctypes.c_void_p(16)
    rc = lib.lm_rhs(ctypes.byref(p), ctypes.c_int64(10), dummy, dummy, ctypes.c_void_p(32),
                    ctypes.c_void_p(48), None)
    assert rc == status
    lib.lm_last_error.restype = ctypes.c_char_p
    assert len(lib.lm_last_error()) > 0


def test_invalid_sizes_and_pointers_rejected(lib):
    p = _params()
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    assert lib.lm_rhs(ctypes.byref(p), ctypes.c_int64(0), a, b, ctypes.c_void_p(48), ctypes.c_void_p(64), None) == -1
    assert lib.lm_rhs(ctypes.byref(p), ctypes.c_int64(5), None, b, ctypes.c_void_p(48), ctypes.c_void_p(64), None) == -1
    # outputs aliasing inputs
    assert lib.lm_rhs(ctypes.byref(p), ctypes.c_int64(5), a, b, a, ctypes.c_void_p(64), None) == -1
    lib.lm_shoot.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lm_shoot(ctypes.byref(p), 5, a, b, 1.0, 0, a, b, None) == -1          # steps < 1
    assert lib.lm_shoot(ctypes.byref(p), 5, a, b, float("inf"), 10, a, b, None) == -1


def test_flow_points_arguments_rejected(lib):
    """Points overlapping the particle buffers, bad sizes and step counts are refused before
    anything is enqueued (fake device addresses: nothing is dereferenced)."""
    P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.lm_flow_points.argtypes = [P, i64, P, P, i64, P, d, i32, P, P, P, P]
    p = _params(dim=2)
    q0, p0, x0 = 0x10000, 0x20000, 0x30000
    call = lambda n, m, x0_, steps, q1, p1, x1, t1=1.0: lib.lm_flow_points(
        ctypes.byref(p), n, q0, p0, m, x0_, t1, steps, q1, p1, x1, None)
    assert call(10, 5, x0, 0, None, None, x0) == -1                  # steps < 1
    assert call(10, 0, x0, 5, None, None, x0) == -1                  # m < 1
    assert call(0, 5, x0, 5, None, None, x0) == -1                   # n < 1
    assert call(10, 5, x0, 5, None, None, None) == -1                # x1 missing
    assert call(10, 5, x0, 5, None, None, q0 + 8) == -1              # x1 inside q0
    assert call(10, 5, p0 + 80, 5, None, None, x0) == -1             # x0 inside p0
    assert call(10, 5, x0, 5, q0 + 8, None, x0) == -1                # q1 overlapping q0, not equal
    assert call(10, 5, x0, 5, None, None, x0, t1=float("nan")) == -1


def test_package_import_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1510_03816_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_one_hip_runtime_whatever_the_import_order(tmp_path):
    """Importing the package before torch must still leave a single HIP runtime in the
    process (the one torch loads): liblm.so binds to it instead of the system copy."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1510_03816_amd\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "print(len(libs)); print(libs)\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.splitlines()
    assert lines[0] == "1", lines


@pytest.mark.parametrize("dtype,cutoff", [(1, 0.0), (0, 0.3)])
def test_autograd_shoot_refuses_unsupported_settings_before_the_shoot(dtype, cutoff):
    """The shooting adjoint exists for double precision with every pair: asking for a gradient
    under single precision or tile skipping fails in the forward pass, before any GPU work
    (the tensors here are host tensors, which the library would reject if it got them)."""
    import torch
    from paper_1510_03816_amd import _lib
    from paper_1510_03816_amd.autograd import shoot
    q = torch.zeros((2, 4), dtype=torch.float64, requires_grad=True)
    p = torch.zeros((2, 4), dtype=torch.float64)
    with pytest.raises(_lib.LmError) as ei:
        shoot(q, p, _params(dtype=dtype, cutoff=cutoff), 1.0, 10)
    assert ei.value.status == _lib.LM_EUNSUPPORTED
