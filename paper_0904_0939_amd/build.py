"""Build libfdtd.so (HIP for gfx950) in-tree.

    python -m paper_0904_0939_amd.build

Compiles csrc/fdtd_step.hip (the fused one-step kernels), csrc/fdtd_step2.hip
(two steps per pass), csrc/fdtd_aux.hip (set-up, upsample, adjoint and
projection kernels) and csrc/fdtd_runtime.cpp with hipcc, in parallel, and
links them into paper_0904_0939_amd/libfdtd.so.  Packed-FP32 instructions are
disabled for every device pass.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfdtd.so")
ARCH = os.environ.get("FDTD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["fdtd_step.hip", "fdtd_step2.hip", "fdtd_aux.hip", "fdtd_runtime.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the library is HIP-only")


def build(verbose: bool = False, jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
    ]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc(), *common, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            for p in procs:
                if p.wait() != 0:
                    raise RuntimeError("hipcc failed")
            procs = []
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SANITIZE_LIB = os.path.join(HERE, "_build", "sanitize", "libfdtd.so")


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime a sanitizer build needs preloaded."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], check=True,
                         capture_output=True, text=True).stdout.strip()
    return out


def build_sanitized(verbose: bool = False) -> str:
    """The host runtime built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host pass only), linked with the regular kernel objects into
    _build/sanitize/libfdtd.so.  For CPU checks of the host code: load it
    with FDTD_LIB_PATH and asan_runtime() preloaded."""
    objdir = os.path.join(HERE, "_build")
    if not all(os.path.exists(os.path.join(objdir, s + ".o")) for s in SOURCES[:-1]):
        build(verbose)
    sdir = os.path.dirname(SANITIZE_LIB)
    os.makedirs(sdir, exist_ok=True)
    obj = os.path.join(sdir, "fdtd_runtime.cpp.o")
    cmd = [hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-x", "hip", "-c",
           os.path.join(CSRC, "fdtd_runtime.cpp"), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    objs = [os.path.join(objdir, s + ".o") for s in SOURCES[:-1]] + [obj]
    subprocess.run([hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", SANITIZE_LIB + ".tmp"],
                   check=True)
    os.replace(SANITIZE_LIB + ".tmp", SANITIZE_LIB)
    return SANITIZE_LIB


if __name__ == "__main__":
    print(build(verbose=True))
