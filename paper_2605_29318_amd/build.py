"""Build libfreeform.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to an object under ``_build/`` in parallel, then hipcc
links the shared library next to this file. The files that decide integers
from floating point (cell index, neighbour predicate) or must match an FP64
reference term by term (shape functions, assembly) build with
-ffp-contract=off; the eigensolver kernels keep contraction on.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfreeform.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = [
    ("ff_ctx.cpp", False),
    ("k_neighbors.hip", True),
    ("k_rkpm.hip", True),
    ("k_assemble.hip", True),
    ("k_lobpcg.hip", False),
    ("k_mlp.hip", False),
    ("k_rowtile.hip", False),
    ("k_paper.hip", True),
    ("k_matfree.hip", False),
    ("k_symspmm.hip", False),
]

COMMON = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-rdc", "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, nocontract: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + COMMON + (["-ffp-contract=off"] if nocontract else []) + [
        "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = list(SOURCES)
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda a: _compile(*a), srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
