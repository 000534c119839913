"""Builds liblbm.so (the HIP kernels and the C ABI of include/lbm.h) for gfx950.

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
for all device code (-packed-fp32-ops).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm.hip")]
HEADERS = [os.path.join(CSRC, h) for h in ("kernels.hpp", "equilibrium.hpp", "equilibrium4.hpp",
                                           "equilibrium13.hpp", "reference49.hpp",
                                           "lattice.hpp")] + \
    [os.path.join(ROOT, "include", "lbm.h")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
         "-I" + os.path.join(ROOT, "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = f"{LIB}.tmp{os.getpid()}"  # unique: parallel builders do not collide
    cmd = [hipcc, *FLAGS, *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
