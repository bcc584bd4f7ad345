"""Builds the HIP library ``librt.so`` (gfx950) in-tree with hipcc.

Every source compiles to its own object in parallel (the FP64 and FP32 step
kernels sit in separate translation units), then one link step makes the
shared library.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# the wave-group step kernels, one unit per precision and groups per wave
# (the largest first, so that the pool overlaps them), then the rest
SOURCES = tuple(f"rt_step3_{p}_g{g}.hip" for g in (4, 3, 2, 1) for p in ("f32", "f64")) + (
    "rt_kernels_f64.hip", "rt_kernels_f32.hip", "rt_api.hip", "rt_serve.hip",
    "rt_quadrature.cpp")
LIB = os.path.join(HERE, "librt.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-value",
]


# Per-file additions (none at present: the backend's iterative
# occupancy-preserving scheduler, once 2 % faster for the FP64 step at four
# waves per SIMD, no longer gains at two and doubles the build time).
EXTRA_FLAGS: dict = {}


def _hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(name: str) -> str:
        obj = os.path.join(OBJDIR, name + ".o")
        cmd = [_hipcc(), *HIPCC_FLAGS, *EXTRA_FLAGS.get(name, []), *inc, "-c",
               os.path.join(CSRC, name), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-lpthread", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
