"""Build libfpo.so (gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 only.  Packed-FP32 instructions are
disabled for device code (-packed-fp32-ops off); hipcc's host pass warns that
it does not know that feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libfpo.so")

SOURCES = [
    "fpo_host.cpp",
    "fpo_render.hip",
    "fpo_train.hip",
    "fpo_bake.hip",
    "fpo_proposal.hip",
    "fpo_construct.hip",
    "fpo_fusion.hip",
    "fpo_occupancy.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        cmd = [HIPCC, "-x", "hip", *DEVICE_FLAGS, "-O3", "-std=c++17", "-fPIC", "-Wall",
               "-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj, *extra]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
