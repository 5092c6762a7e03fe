"""Compile the HIP library ``libhofks.so`` for gfx950 (in-tree)."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "hofks_api.hip")
HEADERS = [os.path.join(PKG, "csrc", h) for h in ("kernels.hpp", "batch.hpp", "closure.hpp", "mlp.hpp", "euler2d.hpp", "kinetic3d.hpp", "kinetic2w.hpp", "weno.hpp", "train.hpp", "probe.hpp", "slope.hpp")] + [
    os.path.join(ROOT, "include", "hofks.h")]
LIB = os.path.join(PKG, "libhofks.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=False):
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
