"""Builds the oracle shared library (plain C, FP64, no contraction of
multiply-adds so that every operation rounds as written)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmosaic_oracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "mosaic_oracle.c")
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-Wextra", "-fPIC", "-shared", "-o", LIB + ".tmp", src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
