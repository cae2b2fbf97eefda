"""Build libgdn.so (the gfx950 HIP library) in-tree with hipcc.

Usage: python -m paper_2512_10386_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgdn.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["frame.hip", "octree.hip", "knn.hip", "score.hip", "dump.hip", "capi.hip", "server.hip", "fit.hip", "eval.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# No FMA contraction anywhere: the fp32 squared distances that decide the
# neighbour sets must round exactly as (dx*dx + dy*dy) + dz*dz. Packed FP32
# instructions are kept off as well.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def source_hash() -> str:
    """SHA-256 over the library's sources (csrc/, include/gdn.h) and compile
    flags. It is compiled into the library (gdn_source_hash) so that a build
    older than its sources is refused when loaded."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    for f in files:
        h.update(f.encode() + b"\0")
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "gdn.h"), "rb") as fh:
        h.update(fh.read())
    # flags without the include path, which depends on where the tree sits
    h.update(" ".join(f for f in FLAGS if not f.startswith(ROOT)).encode())
    return h.hexdigest()


def _compile(src: str, defines=()) -> str:
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = [HIPCC, *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    digest = source_hash()
    defines = {"capi.hip": [f'-DGDN_SOURCE_HASH="{digest}"']}
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines.get(s, ())), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp]
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
