"""Build the decoder library (libpscl.so) for gfx950 with hipcc, in-tree."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libpscl.so")
SOURCES = [os.path.join(CSRC, "decoder.hip"), os.path.join(CSRC, "schedule.cpp"),
           os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "generate.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    # no FMA contraction: G is one rounded add, metric updates one rounded
    # subtraction
    "-ffp-contract=off",
    # no packed-FP32 instruction selection
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build(verbose: bool = False) -> str:
    """Compile every source into LIB_PATH (always recompiles): one object per
    source, in parallel, then one link."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(LIB_DIR, exist_ok=True)
    tag = f".tmp{os.getpid()}"
    objs = [os.path.join(LIB_DIR, os.path.basename(src) + tag + ".o") for src in SOURCES]
    compile_flags = [f for f in FLAGS if f != "-shared"]

    def one(args):
        src, obj = args
        cmd = [HIPCC, *compile_flags, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd).returncode

    try:
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            rcs = list(ex.map(one, zip(SOURCES, objs)))
        if any(rcs):
            raise subprocess.CalledProcessError(max(rcs), "hipcc")
        tmp = LIB_PATH + tag
        cmd = [HIPCC, *FLAGS, *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB_PATH)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
