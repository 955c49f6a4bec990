"""The C-ABI from C: tests/c_abi_host.c, compiled with gcc against
include/heom.h and linked to libheom.so, exercises the host entry points (no
GPU needed)."""
import os
import shutil
import subprocess

import pytest

from paper_1012_4382_amd import heom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_host_entry_points_from_c(tmp_path):
    heom.library()  # raises if libheom.so has not been built
    exe = tmp_path / "c_abi_host"
    lib_dir = os.path.dirname(heom.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_abi_host.c"), "-o", str(exe), "-L", lib_dir, "-lheom",
           f"-Wl,-rpath,{lib_dir}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
