"""Build libns.so (gfx950 only) in-tree with hipcc.

    python -m paper_1201_2118_amd.build

Sources: paper_1201_2118_amd/csrc/*.hip; public header: include/ns.h; kernels
generated from descriptors/kernels.ccl go to _build/gen first.
Objects go to _build/ (not shipped); the library lands next to this file.
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
LIB = os.path.join(PKG, "libns.so")
GEN = os.path.join(BUILD, "gen")

SOURCES = ["kernels.hip", "sor.hip", "sor_fused.hip", "sor_pass.hip", "persist.hip", "generated.hip",
           "adjoint.hip", "runtime.hip"]

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (v_pk_* FP32 forms are avoided)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(c) and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + HIPFLAGS + ["-I", INCLUDE, "-I", CSRC, "-I", GEN, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def generate(verbose: bool = False) -> list:
    """Write the kernels declared in descriptors/kernels.ccl as HIP headers
    into _build/gen (the kernel-descriptor layer; generated.hip includes
    them)."""
    from .descriptors import ccl
    paths = ccl.build(ccl.DESCRIPTOR, GEN)
    if verbose:
        for p in paths:
            print("generated", p, flush=True)
    return paths


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    generate(verbose)
    srcs = list(SOURCES)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
