"""Build the C oracle into ``oracle/libhofks_oracle.so`` with gcc.

Test infrastructure: the shared object is loaded only by the test suite, the
smoke check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hofks_oracle.c")
SOURCES = [SRC, os.path.join(HERE, "mlp_oracle.c")]
LIB = os.path.join(HERE, "libhofks_oracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off keeps every product and sum as written (no fused FMA)
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall",
           "-o", LIB + ".tmp", *SOURCES, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
