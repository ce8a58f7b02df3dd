"""Build ``libshape3d.so`` (the HIP kernels and the C ABI) for gfx950 in-tree.

    python -m paper_2510_02894_amd.build

The marching-cubes table header is regenerated first.  All HIP code is built
with packed FP32 instructions disabled (``-packed-fp32-ops``) and without FMA
contraction, so the FP64 refinement evaluates exactly the operations the
oracle evaluates.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libshape3d.so")
SOURCES = ["mesh.hip", "scan.hip", "pairs.hip", "prune.hip", "soft.hip", "labels.hip", "small.hip", "api.hip"]
# per-file flags: the pair kernels' maxima never see NaNs (MFMA results, or
# FP64 distances of finite positions), so fmax needs no canonicalisation there
EXTRA = {"pairs.hip": ["-fno-honor-nans"], "small.hip": ["-fno-honor-nans"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return [
        "--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-ffp-contract=off", "-mllvm", "-amdgpu-mfma-vgpr-form", "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    ]


def build(verbose: bool = False) -> str:
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_mc_table.py")], check=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC] + flags() + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=%s" % ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
