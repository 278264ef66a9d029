"""Builds the HIP library libnmf_hip.so for gfx950 in-tree with hipcc.

Usage: python -m paper_2101_08431_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnmf_hip.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["anls.hip", "ipm.hip", "dense.hip", "nmf_api.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep packed FP32 instructions out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _stale(src, obj, inc_dirs):
    """True when obj is missing or older than src or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in inc_dirs for f in os.listdir(d) if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose=False, jobs=None, force=True):
    """Compile every source to an object and link the shared library.
    force=False recompiles only objects older than their source or a header."""
    os.makedirs(OBJDIR, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", CSRC, "-I", os.path.join(os.path.dirname(HERE), "include")]

    def compile_one(src):
        obj = os.path.join(OBJDIR, src + ".o")
        if not force and not _stale(os.path.join(CSRC, src), obj, [CSRC, os.path.join(os.path.dirname(HERE), "include")]):
            return obj
        cmd = [hipcc, *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs or min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--changed" not in sys.argv))
