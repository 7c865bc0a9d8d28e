"""Build libaderweno.so (host C++ with g++, kernels with hipcc for gfx950).

Run as ``python -m paper_1408_3719_amd.build`` or through __graft_entry__.build().
The library is written in-tree next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libaderweno.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SOURCES = ["tables.cpp", "topology.cpp", "abi.cpp"]
HIP_SOURCES = ["kernels.hip", "adjoint.hip", "probe.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        # no contraction: the stencil ranking must match an independent
        # implementation bit for bit
        _run(["g++", "-std=c++17", "-O2", "-fPIC", "-pthread", "-ffp-contract=off", "-Wall",
              "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), *inc,
              "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-std=c++17", "-O3",
              "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *inc,
              "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-shared", "-fPIC",
          "-pthread", "-o", tmp, *objs, f"-L{ROCM}/lib", "-lamdhip64"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
