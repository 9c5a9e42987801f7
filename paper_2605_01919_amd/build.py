"""Builds libsdfi.so (all HIP sources, gfx950) next to this file."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsdfi.so")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed float32 instructions anywhere (some forms are unreliable on
    # this hardware); hipcc -O3 would otherwise emit them from plain code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs (no accumulation-register round trip)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _compile(src, verbose):
    obj = os.path.join(HERE, "csrc", os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", *[f for f in FLAGS if f != "-shared"], src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False) -> str:
    # one hipcc per source, several at a time (each is single-threaded)
    srcs = sources()
    workers = max(1, min(len(srcs), (os.cpu_count() or 1), 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        objs = list(pool.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
