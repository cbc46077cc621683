"""Compile the C oracle into ``oracle/libptrt_oracle.so`` with gcc.

Test infrastructure only (see ``oracle/__init__.py``).  Plain ``-O2`` with
OpenMP and no FMA contraction, so the oracle's arithmetic is the arithmetic
written in ``ptrt_oracle.c``; no ``-march=native`` because the library is
built on one host and run on another.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ptrt_oracle.c")
LIB = os.path.join(HERE, "libptrt_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
