"""Compile the gfx950 library ``libswccl.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "swccl.hip"), os.path.join(HERE, "csrc", "server.hip"),
        os.path.join(HERE, "csrc", "cubic.hip")]
LIB = os.path.join(HERE, "libswccl.so")

# -packed-fp32-ops keeps the compiler away from packed fp32 instructions.
HIPFLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    """Always recompile, so a stale library never stands in for the sources."""
    # a fixed temporary name: the compiler records the output path in the
    # library, so a per-process name would make identical sources build differently
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPFLAGS, "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
