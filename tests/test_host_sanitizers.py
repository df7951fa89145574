"""The host set-up code (problem.cpp, algebraic.cpp) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (host code only, no GPU) and
run on structured problems of every kind, their algebraic twins and bad
input (tests/host_sanitize_main.cpp): no sanitizer report, every check
passes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_04356_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-pthread", f"-I{CSRC}",
           os.path.join(CSRC, "problem.cpp"), os.path.join(CSRC, "algebraic.cpp"),
           os.path.join(ROOT, "tests", "host_sanitize_main.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("OK")
