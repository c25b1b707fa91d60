"""Build libcls_hip.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcls_hip.so")

SOURCES = ["cls_track.hip", "cls_quenched.hip", "cls_static.hip", "cls_capi.cpp", "cls_graph.cpp", "cls_autotune.cpp", "cls_server.cpp",
           "cls_quenched_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",          # FP64 arithmetic in the order it is written
    "-munsafe-fp-atomics",        # hardware FP64 atomic add for tallies
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every source into LIB (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *[("-x", "hip", s) if s.endswith(".cpp") else (s,) for s in srcs]]
    flat = []
    for part in cmd:
        if isinstance(part, tuple):
            flat.extend(part)
        else:
            flat.append(part)
    flat += ["-o", tmp]
    if verbose:
        print(" ".join(flat), file=sys.stderr)
    subprocess.check_call(flat)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
