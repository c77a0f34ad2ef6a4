"""The library's host-only code under AddressSanitizer and UBSan: the CSR
checks every entry point runs before device work (validate.h) on valid and
malformed batches held in buffers of exactly their size, and the serving
admission policy (serve_sim.cpp, admission.h) on random arrival traces.
Built with g++ (host code only: no device code is instrumented)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "host_checks")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1812_02091_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
           os.path.join(ROOT, "paper_1812_02091_amd", "csrc", "serve_sim.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host checks ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
