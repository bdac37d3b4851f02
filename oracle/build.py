"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

Compiles kt_oracle.c with gcc into oracle/libkt_oracle.so: FP64, -O2, no FMA
contraction, no fast-math, OpenMP.  No -march=native, so the library runs on
any x86-64 host it is copied to.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kt_oracle.c")
LIB = os.path.join(HERE, "libkt_oracle.so")

CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
