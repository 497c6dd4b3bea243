"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into
libsosfilt.so next to this file (in-tree, so it travels with the sources)."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsosfilt.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (one hipcc each), then
    link the shared library; the library is replaced only on success."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    srcs = sources()
    tmp = LIB + ".tmp%d" % os.getpid()
    with tempfile.TemporaryDirectory(prefix="sosfilt_build_") as d:
        objs = [os.path.join(d, os.path.basename(src) + ".o") for src in srcs]
        cmds = [[hipcc, *flags, *inc, "-c", "-o", o, src] for src, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), file=sys.stderr)
        jobs = max(1, min(len(cmds), os.cpu_count() or 1, 8))
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            for c, rc in zip(cmds, ex.map(subprocess.call, cmds)):
                if rc != 0:
                    raise subprocess.CalledProcessError(rc, c)
        link = [hipcc, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), file=sys.stderr)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
