"""The host code of the library and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

tests/sanitize_host.cpp links the library's host sources (parameter
normalisation, hierarchy enumeration and neighbour tables, the split over
ranks) and the oracle, built with g++ -fsanitize=address,undefined, and runs
them over small systems (N = 1-7, K = 0-2, depth 0-5, at most 3000 ADOs;
plain, scaled and filtered oracle runs).  Any sanitizer report fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_4382_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_host"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I",
           os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "sanitize_host.cpp"), os.path.join(CSRC, "params.cpp"),
           os.path.join(CSRC, "hierarchy.cpp"), os.path.join(CSRC, "shard.cpp"),
           os.path.join(ROOT, "oracle", "heom_oracle.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
