"""The library's host-only code built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, CPU): the stencil description parser on the
test programs and on deterministic mutations of them, and the dense FP64
helpers of Rayleigh-Ritz (tests/sanitize/host_driver.cpp).  Any memory
error, leak or undefined behaviour aborts the driver."""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_09689_amd", "csrc")


def test_parser_and_dense_helpers_under_asan_ubsan(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_driver")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(CSRC, "pv_dsl.cpp"),
           os.path.join(CSRC, "pv_dense.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    progs = sorted(glob.glob(os.path.join(ROOT, "tests", "golden", "dsl", "*.dsl")))
    assert progs
    run = subprocess.run([exe, *progs], env=env, capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "dense helpers ok" in run.stdout
