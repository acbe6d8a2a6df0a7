"""The library's host code (operator-table builders) under AddressSanitizer and
UndefinedBehaviorSanitizer, built for the CPU with g++ (no GPU code involved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_01626_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_operators_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "hostops")
    subprocess.check_call(
        ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I" + CSRC,
         os.path.join(CSRC, "operators.cpp"), os.path.join(ROOT, "tests", "host_ops_driver.cpp"),
         "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe, "12"], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
