"""Builds libheom.so (HIP for gfx950) in place, next to this file.

    python -m paper_1012_4382_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libheom.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -packed-fp32-ops: never emit packed FP32 VALU instructions.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]

SOURCES = ["params.cpp", "hierarchy.cpp", "runtime.cpp", "kernels_dispatch.hip",
           "kernels_lane.hip", "kernels_tile_small.hip", "kernels_tile_7.hip",
           "kernels_tile_8.hip", "kernels_tile_9_10.hip", "kernels_tile_11.hip",
           "kernels_tile_12.hip"]
# The largest translation units first, so the parallel build ends sooner.
_ORDER = ["kernels_tile_12.hip", "kernels_tile_11.hip", "kernels_tile_9_10.hip",
          "kernels_tile_8.hip", "kernels_tile_7.hip"]


def _compile(src: str, defines=(), build_dir: str = BUILD_DIR) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *[f"-D{d}" for d in defines], *lang, "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB, build_dir: str = BUILD_DIR) -> str:
    """Compiles every source and links libheom.so (or `out`); always rebuilds.

    `defines` are extra preprocessor definitions (tuning knobs of the kernels).
    """
    os.makedirs(build_dir, exist_ok=True)
    order = _ORDER + [s for s in SOURCES if s not in _ORDER]
    workers = max(1, min(len(order), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, build_dir), order))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
