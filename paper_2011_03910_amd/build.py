"""Build libjde.so for gfx950 in-tree with hipcc.

Usage: python -m paper_2011_03910_amd.build   (or call build())
"""

import os
import shutil
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libjde.so")
OBJ_DIR = os.path.join(PKG, "_build")

SOURCES = ["conv.hip", "post.hip", "assoc.hip", "ingest.hip", "api.hip", "host_track.cpp"]
ARCH = os.environ.get("JDE_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Wno-unused-lambda-capture"]
# MFMA accumulators stay in ordinary VGPRs: left to its heuristics the compiler
# splits them between VGPRs and AGPRs and copies them back and forth inside the
# K loop (about four copies per MFMA in the implicit GEMM).
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-mllvm", "-amdgpu-mfma-vgpr-form"]


def _hipcc():
    for p in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    raise RuntimeError("hipcc not found: the JDE library needs ROCm's hipcc to build")


def _compile(src):
    out = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [_hipcc(), *HIP_FLAGS, *COMMON, "-x", "hip", "-c", path, "-o", out]
    else:
        cmd = [_hipcc(), *COMMON, "-c", path, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = True) -> str:
    """Compile every source and link libjde.so; returns its path."""
    t0 = time.time()
    os.makedirs(OBJ_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
