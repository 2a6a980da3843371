"""Build libhm.so (gfx950) in-tree.

host.cpp is compiled by g++ with -ffp-contract=off so that the bounding
boxes, midpoints and admissibility tests round like a plain evaluation; the
HIP sources are compiled by hipcc for gfx950 only, with packed FP32 disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# -amdgpu-spill-vgpr-to-agpr=0: the truncation routines are separate functions
# of the persistent executors; letting them park values in accumulation
# registers would count against the register budget of two workgroups per
# compute unit (the executors' launch bound), halving the executors' occupancy.
HIP_FLAGS = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-spill-vgpr-to-agpr=0"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libhm.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in ("host.cpp", "semiauto.cpp"):
        o = os.path.join(BUILD, src.replace(".cpp", ".o"))
        _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall", "-c",
              os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in ("kernels.hip", "capi.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
