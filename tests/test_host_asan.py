"""The library's host code (validation, planning, descriptor building and
their self-checks) built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host side only and driven through its C ABI without a GPU
(tests/asan_host_driver.cpp).  Any out-of-bounds access or use-after-free in
the planner, or undefined arithmetic in its size and offset computations
(signed overflow, out-of-range shifts), fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_10048_amd", "csrc")
from paper_2311_10048_amd.build import SOURCES   # the library's own source list


def test_host_code_under_address_sanitizer():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "drv")
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC]
        cmd += [os.path.join(CSRC, s) for s in SOURCES]
        cmd += [os.path.join(ROOT, "tests", "asan_host_driver.cpp"), "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas",
                "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
        assert b.returncode == 0, b.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
        assert "0 failures" in r.stdout
        assert "AddressSanitizer" not in r.stderr
        assert "runtime error" not in r.stderr
