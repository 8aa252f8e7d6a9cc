"""Build the HIP library liblm.so in-tree for gfx950 (python paper_1510_03816_amd/build.py).

Run it as a script (or through __graft_entry__.build()): importing the package loads the
library, so it cannot be the way to build it.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # packed FP32 instructions stay off: every FP32 operation is a plain VALU op
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 feature and says so; drop that noise
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + out + "\n")
        raise RuntimeError("hipcc failed (exit %d)" % res.returncode)
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source into liblm.so (always recompiles): one object per source,
    compiled in parallel, then one link."""
    import concurrent.futures
    import tempfile
    tmp = LIB + ".tmp%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="liblm_build_") as td:
        objs = [os.path.join(td, os.path.basename(s)[:-4] + ".o") for s in sources()]
        cmds = [[HIPCC] + [f for f in FLAGS if f != "-shared"] + inc + ["-c", "-o", o, s]
                for s, o in zip(sources(), objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            outs = list(ex.map(_run, cmds))
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        outs.append(_run(link))
    if verbose:
        for out in outs:
            if out.strip():
                print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
