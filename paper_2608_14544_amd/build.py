"""Builds libqcl.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2608_14544_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libqcl.so")

SOURCES = ["qcl_api.cpp", "kernels_n2.hip", "kernels_gen2.hip", "kernels_gen3.hip", "kernels_gen4.hip",
           "kernels_gen5.hip", "kernels_gen6.hip", "kernels_gen7.hip", "kernels_gen8.hip",
           "kernels_poly2.hip", "kernels_poly3.hip", "kernels_poly4.hip", "kernels_bil2.hip", "kernels_bil3.hip",
           "kernels_bil4.hip", "kernels_bilh2.hip", "kernels_bilh3.hip", "kernels_bilh4.hip",
           "kernels_bilw2.hip", "kernels_bilw3.hip", "kernels_bilw4.hip", "reduce.hip", "resample.hip",
           "batch_static.hip"]

# Packed-FP32 instructions are disabled on purpose: the step code is
# written in scalar FP32/FP64 and relies on plain IEEE results.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fno-gpu-rdc", "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False, extra=(), jobs: int = 0, only=None) -> str:
    """Compiles every source (in parallel) and links libqcl.so.  ``only``
    restricts compilation to the named sources (the other objects must exist
    from a previous build of the same tree)."""
    from concurrent.futures import ThreadPoolExecutor
    obj_dir = os.path.join(PKG, "_build")
    os.makedirs(obj_dir, exist_ok=True)

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(obj_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc(), *HIP_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    todo = [src for src in SOURCES if only is None or src in only]
    jobs = jobs or min(len(todo) or 1, max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, todo))
    objs = [os.path.join(obj_dir, src + ".o") for src in SOURCES]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"objects missing (build everything once first): {missing}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "-v"]
    build(verbose="-v" in sys.argv, only=args or None)
    print(LIB)
