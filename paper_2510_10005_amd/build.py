"""Build libchem.so (host C++ with the HIP runtime and hipRTC) in-tree, and precompile kernels.

libchem.so holds the mechanism parser, the HIP code generator, the hipRTC driver and the C ABI
of include/chem.h.  The device code is generated per mechanism and compiled for gfx950 by hipRTC;
``precompile`` does that ahead of time for given mechanism files into a kernel cache directory so
that a run on the GPU finds the code objects already built.
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libchem.so")
INCLUDE = os.path.join(ROOT, "include")
KERNEL_CACHE = os.path.join(ROOT, "_build", "kernels")
SOURCES = ["chem.cpp", "codegen.cpp", "mechanism.cpp"]


# HIP flags of device code compiled into the library itself (the allocation-free entry point's
# scratch array); packed FP32 instructions are disabled in every HIP build of this project
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(obj_dir, exist_ok=True)
    dev_obj = os.path.join(obj_dir, "noalloc.o")
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-Wall", "-x", "hip", *DEVICE_FLAGS, "-I", INCLUDE, "-I", CSRC,
           "-c", os.path.join(CSRC, "noalloc.hip"), "-o", dev_obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-Wno-unused-function",
           "-I", INCLUDE, "-I", CSRC, "-o", LIB + ".tmp"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-x", "none", dev_obj]
    cmd += ["-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _precompile_one(job):
    from . import _binding
    path, cache_dir = job
    return _binding.precompile(path, cache_dir)


def precompile(mech_paths, cache_dir: str = KERNEL_CACHE, verbose: bool = True):
    """Generate and hipRTC-compile (gfx950) the kernels of each mechanism file into cache_dir, several
    mechanisms at a time in worker processes (hipRTC compiles of one process do not overlap)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    workers = max(1, min(len(mech_paths), len(os.sched_getaffinity(0)), 16))
    jobs = [(p, cache_dir) for p in mech_paths]
    if workers == 1:
        out = [_precompile_one(j) for j in jobs]
    else:
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as pool:
            out = list(pool.map(_precompile_one, jobs))
    if verbose:
        for p, path in zip(mech_paths, out):
            print(f"precompiled {os.path.basename(p)} -> {path}", flush=True)
    return out


if __name__ == "__main__":
    build_library()
    if len(sys.argv) > 1:
        sys.path.insert(0, ROOT)
        from paper_2510_10005_amd import build as b  # noqa: E402
        b.precompile(sys.argv[1:])
