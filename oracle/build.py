"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libhamls_oracle.so.

Plain C99 + OpenMP, no fused multiply-add contraction, so that the membership
predicate's arithmetic is exactly the written expression.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hamls_oracle.c")
LIB = os.path.join(HERE, "libhamls_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
