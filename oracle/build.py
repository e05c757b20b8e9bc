"""Build the FP64 CPU oracle (test infrastructure) into oracle/libpmoracle.so.

Plain gcc, IEEE arithmetic: -O2 -fno-fast-math -ffp-contract=off (no fused
multiply-add contraction), OpenMP over rows only (each node is independent,
so threading does not change any result).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmoracle.c")
LIB = os.path.join(HERE, "libpmoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
