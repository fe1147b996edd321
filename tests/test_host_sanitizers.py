"""Host-only library code under the address and undefined-behaviour sanitizers.

tests/fuzz_host.cpp drives the tuning-cache parser (malformed, mutated and
random text; file round trip), the cache key and the plan-time validation of
random problems. It is compiled with g++ together with the library's
host-only source (no device code is involved) and must finish without a
sanitizer report.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_host_logic_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "fuzz_host")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "fuzz_host.cpp"),
           os.path.join(ROOT, "paper_1210_2687_amd", "csrc", "admm_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "0 failures" in r.stdout
