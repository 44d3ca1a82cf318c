"""Build libosm.so in-tree for gfx950 with hipcc (one object per source,
compiled in parallel, then linked)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libosm.so")
SOURCES = ["osm.hip", "kernels_assemble.hip", "kernels_factor.hip", "kernels_solve.hip",
           "kernels_control.hip", "kernels_batch.hip", "kernels_net.hip",
           "kernels_gmres.hip", "kernels_krylov.hip", "kernels_pade.hip", "kernels_yorder.hip",
           "kernels_lhmodal.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -simplifycfg-sink-common=false: the IR-level sinking of identical
# instructions from several predecessors once merged the last store of two
# call sites of a row-finishing routine (the one in registers and the one
# streamed in a loop); the AMDGPU structurizer then ran the loop's wave sums
# (DPP moves and lane reads, which need every lane active) with the lane
# that owed the merged store masked off, and the solve returned non-finite
# values.  tests/test_solve_codegen.py checks the generated code for it.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-simplifycfg-sink-common=false",
         "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
