"""Build libedm.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2105_12301_amd.build   (or call build()).
Every source is compiled on every call; objects go to ``_build/``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libedm.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("EDM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["edm_api.hip", "knn.hip", "sweep_multi.hip", "gram.hip", "fixup.hip", "lookup.hip", "misc.hip", "net.hip", "plan.hip", "twokernel.hip", "subsample.hip", "noalloc.hip", "ceilings.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are not used anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]
# Per-file extras: the neighbour key must be evaluated without contraction.
EXTRA = {"knn.hip": ["-ffp-contract=off"], "sweep_multi.hip": ["-ffp-contract=off"], "gram.hip": ["-ffp-contract=off"], "fixup.hip": ["-ffp-contract=off"],
         "twokernel.hip": ["-ffp-contract=off"],
         "subsample.hip": ["-ffp-contract=off"]}


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libedm)")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc(), *COMMON, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libedm.so failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
