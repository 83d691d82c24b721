"""Build the HIP library (libmls_hip.so) in-tree for gfx950.

Every .hip and .cpp file under csrc/ is compiled with hipcc and linked into
one shared library next to this file.  The build always recompiles (it is
the "does it build" check as well as the build).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmls_hip.so")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # keep the compiler from emitting packed float32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, defines=()) -> str:
    cmd = [_hipcc(), *COMMON, *[f"-D{d}" for d in defines],
           "-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str | None = None, defines=(), srcdir: str | None = None) -> str:
    """Compile and link; ``out``, ``defines`` (extra -D flags) and ``srcdir``
    serve variant builds outside the tree."""
    src_root = srcdir or CSRC
    srcs = sorted(glob.glob(os.path.join(src_root, "*.hip")) + glob.glob(os.path.join(src_root, "*.cpp")))
    lib = out or LIB
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    workers = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        for o in ex.map(lambda s_o: _compile(*s_o, defines), zip(srcs, objs)):
            if verbose:
                print("compiled", os.path.basename(o))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
