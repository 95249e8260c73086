"""Build the gfx950 shared library ``libctcsgd.so`` in-tree with hipcc.

    python -m paper_1709_00953_amd.build

Every call recompiles.  All HIP code is built with packed-FP32 instruction
selection disabled (``-Xclang -target-feature -Xclang -packed-fp32-ops``);
the kernel file also with ``-fno-honor-nans``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libctcsgd.so")
ARCH = os.environ.get("CT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    common = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src, lang in (("ct_kernels.hip", "hip"), ("ct_api.cpp", "hip"), ("ct_server.cpp", "hip")):
        obj = os.path.join(bdir, src + ".o")
        cmd = [cc, "-x", lang, "-c", os.path.join(CSRC, src), "-o", obj] + common
        if src == "ct_kernels.hip":
            # the kernels never produce or test NaNs: min/max need no
            # canonicalising of their operands (the host code, which checks
            # descriptions for NaN, is built without this)
            cmd.append("-fno-honor-nans")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
