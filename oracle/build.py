"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP for the update and upsample sweeps only.  Used by the test
suite, the smoke check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdtd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


SANITIZE_LIB = os.path.join(HERE, "_sanitize", "liboracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    """AddressSanitizer + UndefinedBehaviorSanitizer build (clang, the same
    sanitizer runtime as the library's sanitizer build; serial: no OpenMP).
    Load it with FDTD_ORACLE_LIB and the clang ASan runtime preloaded."""
    os.makedirs(os.path.dirname(SANITIZE_LIB), exist_ok=True)
    cmd = [CLANG, "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", SRC,
           "-o", SANITIZE_LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(SANITIZE_LIB + ".tmp", SANITIZE_LIB)
    return SANITIZE_LIB


if __name__ == "__main__":
    print(build(verbose=True))
