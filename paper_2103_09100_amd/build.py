"""Compile the C-ABI library ``libsbfem.so`` for gfx950 with hipcc (in-tree).

Run ``python -m paper_2103_09100_amd.build``.  Each translation unit is
compiled in parallel into ``_build/`` and linked next to this file, where the
binding loads it.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsbfem.so")
SOURCES = ["kernels.hip", "mixed_ebe_fp64.hip", "mixed_ebe_fp32.hip", "mixed_tiled_fp64.hip",
           "mixed_tiled_fp32.hip", "mixed_tiled_fp64r.hip", "mixed_tiled_fp32r.hip", "mixed_hang_mma_fp64.hip",
           "mixed_hang_mma_fp32.hip", "mixed_hang_mma_fp16.hip", "mixed_hang_mma_bf16.hip", "owner_fp64.hip", "owner_fp32.hip",
           "owner_fp16.hip", "owner_bf16.hip", "linalg.hip", "sbfem.cpp", "tiling.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # packed FP32 instructions stay off (their results were unreliable on these boxes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 subnormals flushed to zero: a wave front started from rest carries values far
    # below 1e-38 that are irrelevant to the result but slow FP32 LDS arithmetic down
    "-fgpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function",
]


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{msg}")
    if msg.strip() and verbose:
        print(msg, flush=True)
    return obj


def build(verbose=True):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
