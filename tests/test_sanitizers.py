"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library's host runtime and the FP64 oracle are rebuilt with both
sanitizers, and the C-ABI contract tests and the oracle pins run against those
builds in a child process with the sanitizer runtime preloaded.  Any report
(out-of-bounds access, use after free, undefined behaviour) aborts the child
and fails the test.  No GPU is used: without one every device call of the
library returns FDTD_EHIP before touching device memory."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_and_oracle_pins_are_clean_under_asan_and_ubsan():
    from oracle import build as obuild
    from paper_0904_0939_amd import build as lbuild

    lib = lbuild.build_sanitized()
    olib = obuild.build_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": lbuild.asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "FDTD_LIB_PATH": lib,
        "FDTD_ORACLE_LIB": olib,
        "HIP_VISIBLE_DEVICES": "",  # host code only, also on a machine with a GPU
    })
    # the sanitizer runtime is really there in the child
    probe = [sys.executable, "-c", "import ctypes; ctypes.CDLL(None).__asan_report_load8"]
    assert subprocess.run(probe, env=env, capture_output=True).returncode == 0
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "tests/test_abi_cpu.py", "tests/test_oracle_pins.py", "tests/test_oracle_potential_pins.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
