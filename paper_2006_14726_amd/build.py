"""Build the gfx950 HIP library libsplat.so in-tree with hipcc.

Every source is compiled to its own object in parallel (each kernel is
launched from the file that defines it, so no device linking is needed),
then the objects are linked into one shared library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsplat.so")
SOURCES = ["api.hip", "unproject.hip", "bvh.hip", "trace.hip", "schedule.hip", "march.hip", "codec.hip", "accum.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions: they have miscomputed on these parts
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every csrc/*.hip and link them into one shared library; raises on failure."""
    include = os.path.join(os.path.dirname(HERE), "include")
    with tempfile.TemporaryDirectory(prefix="splat_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [["hipcc", *FLAGS, "-I", include, *(extra or []), "-c", "-o", o, os.path.join(CSRC, s)]
                for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), file=sys.stderr)
        jobs = min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16)
        with ThreadPoolExecutor(max_workers=max(jobs, 1)) as pool:
            for f in [pool.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = out + ".tmp"
        link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), file=sys.stderr)
        subprocess.check_call(link)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
