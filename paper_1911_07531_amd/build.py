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
# -amdgpu-spill-vgpr-to-agpr=0 and -amdgpu-mfma-vgpr-form: the truncation
# routines are separate functions of the persistent executors; letting them
# park values in, or keep matrix-core accumulators in, accumulation registers
# counts against the register budget of two workgroups per compute unit (the
# executors' launch bound) and halves the executors' occupancy.
HIP_FLAGS = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-spill-vgpr-to-agpr=0", "-mllvm", "-amdgpu-mfma-vgpr-form"]
# executors whose occupancy must stay at two waves per SIMD (two workgroups per CU)
EXECUTORS = ("exec_dataflow_kernel", "exec_level_kernel", "fused_dataflow_kernel")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def _check_occupancy(remarks: str) -> None:
    """Fail the build when an H-LU executor kernel fits fewer than two waves per
    SIMD (the compiler's resource-usage remarks), i.e. one workgroup per CU."""
    name = None
    for line in remarks.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split()[0]
        elif "Occupancy [waves/SIMD]:" in line and name and any(e in name for e in EXECUTORS):
            occ = int(line.split("Occupancy [waves/SIMD]:")[1].split()[0])
            if occ < 2:
                raise RuntimeError(f"{name}: occupancy {occ} wave(s) per SIMD, the executors need 2")


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
        extra = ["-Rpass-analysis=kernel-resource-usage"] if src == "kernels.hip" else []
        r = _run([HIPCC, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o])
        if extra:
            _check_occupancy(r.stderr)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
