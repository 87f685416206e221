"""Compile the C oracle into ``oracle/liboracle.so`` with gcc.

The oracle is test infrastructure: a plain single-threaded C implementation
checked against the paper.  It is built with -O2, no fast-math and no FMA
contraction, so its binary64 threshold arithmetic follows the source exactly.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sfgen_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
        "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
