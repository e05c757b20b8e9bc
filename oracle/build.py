"""Build the FP64 CPU oracle (test infrastructure) into oracle/libpmoracle.so.

Plain gcc, IEEE arithmetic: -O2 -fno-fast-math -ffp-contract=off (no fused
multiply-add contraction), OpenMP over rows only (each node is independent,
so threading does not change any result).

``python oracle/build.py --sanitize`` builds the same library with
AddressSanitizer and UndefinedBehaviorSanitizer (any report aborts); run the
CPU tests against it with the gcc ASan runtime preloaded:

    python oracle/build.py --sanitize
    LD_PRELOAD=$(gcc -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0 \\
        UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 python -m pytest tests -m "not gpu"
    python oracle/build.py            # back to the plain build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pmoracle.c")
LIB = os.path.join(HERE, "libpmoracle.so")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra"] + (SANITIZE if sanitize else []) + [
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
