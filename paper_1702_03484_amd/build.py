"""Build libmapsq.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled with hipcc into _build/, then linked
into paper_1702_03484_amd/libmapsq.so.  ``build()`` always recompiles.
``build(debug=True)`` (``python -m paper_1702_03484_amd.build --debug``)
compiles the same sources with -DMQ_DEBUG into _build_debug/ and links
libmapsq_debug.so: the bounds-checked build, loaded by the binding when
MAPSQ_LIB=debug.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmapsq.so")
BUILD_DEBUG = os.path.join(HERE, "_build_debug")
LIB_DEBUG = os.path.join(HERE, "libmapsq_debug.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["k_sort.hip", "k_reduce.hip", "k_map.hip", "k_util.hip", "k_batch.hip", "k_semi.hip", "k_merge.hip", "noalloc.hip", "k_dict.hip", "dict.cpp", "runtime.cpp", "arena.cpp", "planner.cpp",
           "batch.cpp", "serve.cpp", "capi.cpp"]
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(os.path.dirname(HERE), "include"),
]


def _compile(src: str, debug: bool = False) -> str:
    obj = os.path.join(BUILD_DEBUG if debug else BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DMQ_DEBUG"] if debug else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
    if errs:
        print(errs, file=sys.stderr)
    return obj


def build(jobs: int = 8, debug: bool = False) -> str:
    os.makedirs(BUILD_DEBUG if debug else BUILD, exist_ok=True)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, debug), SOURCES))
    lib = LIB_DEBUG if debug else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(debug="--debug" in sys.argv[1:]))
