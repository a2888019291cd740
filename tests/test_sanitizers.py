"""AddressSanitizer + UndefinedBehaviorSanitizer (+ LeakSanitizer at exit) over the CPU
code: the C oracle's every entry point (tests/sanitize/oracle_driver.c) and the library's
host-side math, i.e. the prime chain, Philox, secret, slot encoding, guess and scaled
plan, the bootstrap's planning and the learned guess's file form
(tests/sanitize/host_driver.cpp).  Each driver is
compiled with gcc/g++ and the sanitizers, run, and must exit 0 with no report.  The
GPU code is not built here (no device sanitizer runs on this hardware)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _run(cmd_build, exe, cwd=None):
    r = subprocess.run(cmd_build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300, cwd=cwd)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    out = _run(["gcc", *SAN, "-std=gnu11", "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                os.path.join(ROOT, "oracle", "ckks_oracle.c"), "-o", exe, "-lm"], exe)
    assert "oracle driver: ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not available")
def test_host_math_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_driver")
    csrc = os.path.join(ROOT, "paper_2509_08383_amd", "csrc")
    out = _run(["g++", *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + csrc,
                os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(csrc, "host_math.cpp"),
                os.path.join(csrc, "boot_plan.cpp"), os.path.join(csrc, "mlp_file.cpp"), "-o", exe], exe, cwd=str(tmp_path))
    assert "host driver: ok" in out
