"""Build libbtpcg.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2503_15269_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbtpcg.so")
ARCH = os.environ.get("BTPCG_ARCH", "gfx950")

SOURCES = ["api.cpp", "setup.hip", "solve.hip", "solve_fast.hip",
           "solve_fast24.hip", "mrhs.hip", "direct.hip", "grid.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed float32 vector instructions stay off (see DESIGN notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


# Per-source flags. The register-resident batch kernel runs at two
# wavefronts per SIMD and is bound by instruction issue and latency; LLVM's
# iterative ILP scheduling strategy orders the inner loop of its n = 12
# variants better than the default (batch solve 0.94 -> 0.91 ms on gfx950,
# same arithmetic) but that of the n = 24 variant worse (0.64 -> 0.83 ms),
# which is therefore built in solve_fast24.hip with the default. It also
# shortens the direct solver's dependent chains a little (n = 48: 3 %); the
# other sources gain nothing from it.
_ILP = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]
SOURCE_FLAGS = {"solve_fast.hip": _ILP, "direct.hip": _ILP}


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(c) and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    cmd += FLAGS + SOURCE_FLAGS.get(os.path.basename(src), [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp]
    cmd += objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
