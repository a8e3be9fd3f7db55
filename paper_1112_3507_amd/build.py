"""Build libhp.so (HIP, gfx950) in-tree: ``python -m paper_1112_3507_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = ["csrc/hp_kernels.hip", "csrc/hp_solver.hip", "csrc/hp_nn.hip", "csrc/hp_noalloc.hip", "csrc/hp_hydro.hip",
           "csrc/hp_fcg.hip", "csrc/hp_coarse.hip"]
LIB = os.path.join(PKG, "libhp.so")
ARCH = "gfx950"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libhp.so (always recompiles)."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(PKG, "csrc", os.path.basename(src) + ".o")
        cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-c",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               "-I", os.path.join(ROOT, "include"), "-o", obj, os.path.join(PKG, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
