"""Build libsfa.so (host compiler + HIP runtime and kernels) for gfx950, in-tree.

Every source compiles to an object of its own, in parallel (the walk kernels
are instantiated in one translation unit per stride or id width), and hipcc
links the objects into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfa.so")

HOST_SOURCES = ["compiler.cpp"]
HIP_SOURCES = [
    "runtime.hip", "batch.hip", "stream.hip",
    "walk_lds_s1.hip", "walk_lds_s2.hip", "walk_lds_s4.hip",
    "walk_global_u8.hip", "walk_global_u16.hip", "walk_global_u32.hip", "walk_partial.hip",
    "walk_partial_vector.hip", "walk_vector.hip",
]
BUILD_DIR = os.path.join(HERE, "_build")
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the walk loops are unrolled in full (ring buffers indexed by constants
    # stay in registers); the global-table walk's body exceeds the default
    # limit for such loops
    "-mllvm", "-pragma-unroll-threshold=1000000",
    "-Wall", "-Wno-unused-result",
]


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit():
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmds = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    # longest first: the walk instantiations dominate
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        list(ex.map(run, sorted(cmds, key=lambda c: "walk_" not in c[-3])))
    tmp = LIB + ".tmp"
    run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
