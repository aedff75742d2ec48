"""Compile the HIP sources of libmd for gfx950 into paper_1105_5613_amd/libmd.so.

Every translation unit is compiled with hipcc -O3 for gfx950 only, with the
packed-FP32 instructions disabled; the neighbour search additionally with
-ffp-contract=off (its inclusion test must round exactly like a plain FP64
evaluation).  Objects go to _build/ in the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmd.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-x", "hip",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Werror", "-Wno-unused-command-line-argument",
          "-I", os.path.join(HERE, "..", "include")]
PER_FILE = {"nlist.hip": ["-ffp-contract=off"], "nlist_small.hip": ["-ffp-contract=off"],
            "analysis.hip": ["-ffp-contract=off"]}
SOURCES = ["cells.hip", "nlist.hip", "nlist_small.hip", "force.hip", "force_staged.hip", "force_cells.hip",
           "integrate.hip", "analysis.hip", "md_api.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *PER_FILE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
