"""Build step for the CPU oracle (test infrastructure, not the product).

Compiles ``mtpt_oracle.c`` into ``libmtpt_oracle.so`` next to it with gcc,
FP contraction off so that every arithmetic operation in the source is one
IEEE-rounded operation, and OpenMP for the per-particle loops.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mtpt_oracle.c")
LIB = os.path.join(HERE, "libmtpt_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile the oracle library; returns its path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
