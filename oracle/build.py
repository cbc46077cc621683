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


FLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
         "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc"] + FLAGS + ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_variant(replacements, out_dir: str) -> str:
    """Compile a copy of the oracle with each (old, new) text replacement
    applied (every `old` must occur exactly once) into out_dir; returns the
    library path.  Used only by the tests that plant a mistake in the oracle
    and check that its pins catch it."""
    with open(SRC) as fh:
        text = fh.read()
    for old, new in replacements:
        if text.count(old) != 1:
            raise ValueError(f"replacement target must occur once: {old!r}")
        text = text.replace(old, new)
    src = os.path.join(out_dir, "ptrt_oracle_variant.c")
    lib = os.path.join(out_dir, "libptrt_oracle_variant.so")
    with open(src, "w") as fh:
        fh.write(text)
    subprocess.run(["gcc"] + FLAGS + ["-o", lib, src, "-lm"], check=True)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
