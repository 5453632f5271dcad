"""Builds the package's native libraries in-tree.

libgraphgen.so -- seeded input generators (host C++, g++).
libblest.so    -- the BVSS BFS library: host runtime + gfx950 HIP kernels (hipcc).
"""
from __future__ import annotations

import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# Packed-FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-munsafe-fp-atomics"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_graphgen(verbose: bool = False) -> str:
    src = os.path.join(PKG, "inputs", "graphgen.cpp")
    out = os.path.join(PKG, "inputs", "libgraphgen.so")
    _run(["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread", "-Wall", src, "-o", out + ".tmp"], verbose)
    os.replace(out + ".tmp", out)
    return out


def build_blest(verbose: bool = False, jobs: int = 8) -> str:
    out = os.path.join(PKG, "libblest.so")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objs, procs = [], []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = [hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", s, "-o", o]
        if s.endswith(".cpp"):
            cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-I", INCLUDE, "-I", CSRC,
                   "-D__HIP_PLATFORM_AMD__", "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("compile failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed")
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", out + ".tmp"], verbose)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> None:
    build_graphgen(verbose)
    build_blest(verbose)


if __name__ == "__main__":
    build(verbose=True)
