"""Build libflb.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1204_6734_amd.build        # or build() from Python

Every HIP source is compiled with packed-FP32 instruction selection turned
off (those instructions are not used by this library), and with
multiply-adds fused only where one source expression holds both
(-ffp-contract=on): the rounding of every result is then fixed by the
source, so the kernel variants that share the collision (with and without
the correlator sums, for instance) produce bit-identical populations.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libflb.so")

SOURCES = ["flb_step.hip", "flb_kernels.hip", "flb_d3q19.hip", "flb_noalloc.hip", "flb_runtime.cpp",
           "flb_group.cpp", "flb_server.cpp", "flb_tune.cpp", "flb_d3q19.cpp"]
ARCH = os.environ.get("FLB_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libflb")
    return exe


def compile_flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=on", "-munsafe-fp-atomics", "-I", INCLUDE, "-I", CSRC,
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    """Compile every source to an object file, then link libflb.so."""
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *compile_flags(), *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
