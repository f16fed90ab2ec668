"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(CPU only): the oracle's C filters, and the library's host source (with its
device code compiled as usual, the sanitizers on the host side only), each
linked into a small driver that exercises them on random and edge inputs
(tests/sanitize/).  A sanitizer report or a failed expectation ends the
driver with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1707_09683_amd", "csrc")
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(exe, env=ENV):
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, f"{exe}: status {p.returncode}\n{p.stdout[-2000:]}\n{p.stderr[-4000:]}"
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-4000:]
    return p.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-pthread", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "filters.c"),
                    os.path.join(ROOT, "oracle", "p7viterbi.c"),
                    os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"],
                   check=True, capture_output=True, timeout=600)
    assert "oracle driver done" in _run(exe)


def test_host_library_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_driver")
    cmd = [hipcc, "-O1", "-g", "-std=c++20", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-Wno-unused-command-line-argument",
           "-x", "hip", os.path.join(CSRC, "hmsv_host.cpp"), os.path.join(CSRC, "select.hip"),
           os.path.join(SAN, "host_driver.cpp"), "-o", exe]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert p.returncode == 0, p.stderr[-4000:]
    # the HIP runtime's own allocations outlive main: leak checks off here
    env = {**ENV, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0"}
    assert "host driver done" in _run(exe, env)
