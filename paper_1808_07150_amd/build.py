"""Build libspdhg.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libspdhg.so")
SOURCES = [os.path.join(HERE, "csrc", "spdhg.hip"), os.path.join(HERE, "csrc", "convnet.hip")]
DEPENDS = SOURCES + [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "geom.hpp")] + \
    [os.path.join(ROOT, "include", h) for h in ("spdhg.h", "spdhg_net.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # no FMA contraction: fused multiply-adds are written out where wanted, so the forward
    # walk and the gather backprojector evaluate identical expressions
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (each carries its own gfx950 code
    object), then link the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = f".tmp{os.getpid()}"
    objs = [os.path.join(HERE, "csrc", os.path.basename(src) + tag + ".o") for src in SOURCES]
    procs = []
    for src, obj in zip(SOURCES, objs):
        cmd = [hipcc] + [f for f in HIPCC_FLAGS if f != "-shared"] + \
            ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                      text=True))
    failed = False
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out)
            failed = True
    try:
        if failed:
            raise RuntimeError("hipcc failed building libspdhg.so")
        tmp = LIB + tag
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking libspdhg.so failed")
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(f) <= t for f in DEPENDS)


if __name__ == "__main__":
    print(build(verbose=True))
