"""Compile the CPU oracle (test infrastructure) into oracle/libmpk_oracle.so.

The flags keep binary64 semantics plain: no FMA contraction, no fast-math,
round-to-nearest-even; fma() is only used where the source calls it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpk_oracle.c")
LIB = os.path.join(HERE, "libmpk_oracle.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized"]


def build(verbose=False):
    cmd = ["gcc"] + CFLAGS + ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
