"""Compile the CPU oracle (plain C, FP64, OpenMP) into oracle/libucp_oracle.so.

Test infrastructure: the oracle is only ever loaded by the test suite, the
smoke check and the benchmark's CPU-baseline leg.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ucp_oracle.c")
LIB = os.path.join(HERE, "libucp_oracle.so")

# -ffp-contract=off: no fused multiply-adds beyond the explicit fma() calls, so
# the opening test and the key quantisation are evaluated exactly as written.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
