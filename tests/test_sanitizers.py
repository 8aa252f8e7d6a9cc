"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

- The oracle (oracle/lm_oracle.c), built with gcc's sanitizers and driven by
  tests/sanitize/oracle_check.c over every oracle function on small and ragged inputs.
- The host side of the C ABI: the library's sources built with the sanitizers on their host
  code only (device code unchanged), driven by tests/sanitize/abi_check.c through argument
  validation of every entry point and the host-only planners.  Nothing reaches a GPU.

A sanitizer report makes the driver exit non-zero (no recovery), which fails the test.
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1510_03816_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert out.returncode == 0, "%s\n%s" % (" ".join(cmd), out.stdout[-4000:])
    return out.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", "-o", exe,
          os.path.join(HERE, "oracle_check.c"), os.path.join(ROOT, "oracle", "lm_oracle.c"), "-lm"])
    out = _run([exe], env=SAN_ENV, timeout=300)
    assert "ok" in out and "runtime error" not in out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs the ROCm compilers")
def test_c_abi_host_side_under_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", INCLUDE]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [str(tmp_path / (os.path.basename(s)[:-4] + ".o")) for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda so: _run([HIPCC, "-c"] + common + san + ["-o", so[1], so[0]]), zip(srcs, objs)))
    lib = str(tmp_path / "liblm_san.so")
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + san + ["-o", lib] + objs)
    exe = str(tmp_path / "abi_check")
    _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", INCLUDE,
          os.path.join(HERE, "abi_check.c"), "-L", str(tmp_path), "-llm_san", "-Wl,-rpath," + str(tmp_path),
          "-o", exe])
    out = _run([exe], env=SAN_ENV, timeout=300)
    assert "ok" in out and "runtime error" not in out
    shutil.rmtree(tmp_path, ignore_errors=True)
