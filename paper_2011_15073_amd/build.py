"""Build the gfx950 HIP library libpmlbm.so in-tree (hipcc, no JIT cache).

All HIP code is compiled with packed-FP32 instruction selection disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host pass warns
that it does not know the feature, which is harmless.

``-ffp-contract=on`` fuses a*b+c only inside one source expression, so the
rounding of every operation is fixed by the source and not by how a kernel
inlines, peels or unrolls it: the batched-sweep kernel and the single-case
kernel, which share the per-node code, then round identically.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmlbm.so")
SOURCES = ["pm_kernels.hip", "pm_adjoint.hip", "pm_api.hip"]
ARCH = os.environ.get("PMLBM_ARCH", "gfx950")


# Host-code sanitizers (AddressSanitizer and UndefinedBehaviorSanitizer on the
# host pass only; device code is built as usual): ``python build.py
# --sanitize-host``, then run the CPU tests with clang's ASan runtime preloaded,
#   LD_PRELOAD=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so) \
#   ASAN_OPTIONS=detect_leaks=0 python -m pytest tests/test_abi.py
# and rebuild without the option afterwards.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, sanitize_host: bool = False) -> str:
    cmd = ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
           "-ffp-contract=on",
           "-shared", "-Wall", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp"] + (HOST_SANITIZE if sanitize_host else []) + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize_host="--sanitize-host" in sys.argv))
