"""The plan-time host code (nested SVD by one-sided Jacobi, sinc quadrature,
circulant columns, B-spline moduli) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU over cubic, non-cubic, odd,
full-rank and Lagrange cases (tests/host_sanitize_driver.cpp).  Host code
only: no device code is compiled or run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_18838_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_factor_construction_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
           os.path.join(HERE, "host_sanitize_driver.cpp"), os.path.join(CSRC, "factors.cpp"),
           os.path.join(CSRC, "quadrature.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok"), r.stdout[-2000:]
