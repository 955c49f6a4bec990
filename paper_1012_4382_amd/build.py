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

# FP64 tile kernels take their arguments preloaded into scalar registers
# (gfx950 kernel-argument preloading), which removes one dependent scalar load
# from the start of every workgroup: 2.5-3.5 % faster per stage on the FP64
# shapes, 1-4 % slower on the FP32-mixed ones, which are built without it.
TILE_F64_FLAGS = ["-mllvm", "-amdgpu-kernarg-preload-count=8"]

# (source, tile launch shape, tile storage is FP64) for the tile units; None
# for the others.  The tile units of N <= 8 are compiled once per shape (the
# autotuner's candidates) and N = 9..12 in the default shape only, each once
# per storage precision.
_SHAPES = 5
SOURCES = ([("params.cpp", None, None), ("hierarchy.cpp", None, None),
            ("runtime.cpp", None, None), ("autotune.cpp", None, None), ("shard.cpp", None, None),
            ("kernels_dispatch.hip", None, None), ("kernels_lane.hip", None, None)] +
           [(f"kernels_tile_{u}.hip", s, f64) for u in ("small", "7", "8")
            for s in range(_SHAPES) for f64 in (True, False)] +
           [(f"kernels_tile_{u}.hip", 0, f64) for u in ("9_10", "11", "12")
            for f64 in (True, False)])
# The largest translation units first, so the parallel build ends sooner.
_FIRST = ["kernels_tile_12.hip", "kernels_tile_11.hip", "kernels_tile_9_10.hip",
          "kernels_tile_8.hip", "kernels_tile_small.hip", "kernels_tile_7.hip"]


def _newest_input(src: str) -> float:
    """Modification time of a source and of every header it can include."""
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    heads += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return max(os.path.getmtime(p) for p in [os.path.join(CSRC, src), __file__, *heads])


def _compile(unit, defines=(), build_dir: str = BUILD_DIR, incremental: bool = False) -> str:
    src, shape, f64 = unit
    stem = os.path.basename(src) + ("" if shape is None else f".s{shape}.f{int(f64)}")
    obj = os.path.join(build_dir, stem + ".o")
    if (incremental and not defines and os.path.exists(obj) and
            os.path.getmtime(obj) > _newest_input(src)):
        return obj
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    extra = [] if shape is None else [f"-DHEOM_SHAPE={shape}", f"-DHEOM_TILE_F64={int(f64)}"]
    if f64:
        extra += TILE_F64_FLAGS
    cmd = [HIPCC, *COMMON, *[f"-D{d}" for d in defines], *extra, *lang, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB, build_dir: str = BUILD_DIR,
          incremental: bool = False) -> str:
    """Compiles every source and links libheom.so (or `out`); rebuilds every
    object unless `incremental` (then only objects older than their source, a
    header or this script).

    `defines` are extra preprocessor definitions (tuning knobs of the kernels).
    """
    os.makedirs(build_dir, exist_ok=True)
    order = sorted(SOURCES, key=lambda u: _FIRST.index(u[0]) if u[0] in _FIRST else len(_FIRST))
    workers = max(1, min(len(order), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, build_dir, incremental), order))
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
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
