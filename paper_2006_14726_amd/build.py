"""Build the gfx950 HIP library libsplat.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsplat.so")
SOURCES = ["api.hip", "unproject.hip", "bvh.hip", "trace.hip", "schedule.hip", "march.hip", "codec.hip", "accum.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions: they have miscomputed on these parts
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every csrc/*.hip into one shared library; raises on failure."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    include = os.path.join(os.path.dirname(HERE), "include")
    cmd = ["hipcc", *FLAGS, "-I", include, *(extra or []), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
