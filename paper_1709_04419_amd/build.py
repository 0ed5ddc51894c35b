"""Builds libhmlik.so (the HIP library behind include/hmlik.h) in-tree for gfx950.

    python -m paper_1709_04419_amd.build

Host planner code is compiled without floating-point contraction so that
the cluster tree and the admissibility partition are reproducible bit for
bit; device code is compiled for gfx950 with packed-FP32 instructions
disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhmlik.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build_library(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    # host planner: exact, no contraction
    o = os.path.join(BUILD, "hm_plan.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", *inc, "-c",
          os.path.join(CSRC, "hm_plan.cpp"), "-o", o])
    objs.append(o)
    # host API
    o = os.path.join(BUILD, "hm_api.o")
    _run([HIPCC, "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", *inc, "-c",
          os.path.join(CSRC, "hm_api.cpp"), "-o", o])
    objs.append(o)
    # request server
    o = os.path.join(BUILD, "hm_server.o")
    _run([HIPCC, "-O2", "-std=c++17", "-fPIC", *inc, "-c",
          os.path.join(CSRC, "hm_server.cpp"), "-o", o])
    objs.append(o)
    # device kernels
    o = os.path.join(BUILD, "hm_device.o")
    _run([HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", *inc,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-c", os.path.join(CSRC, "hm_device.hip"), "-o", o])
    objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
