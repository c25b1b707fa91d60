"""Instruction-rate microbenchmarks on the GPU (issue rates behind the VALU work model).

Builds csrc/microbench.hip into libcls_microbench.so on first use and reports, per
operation, the measured lane-operations per second and that rate as a fraction
of the full-rate VALU peak (256 CUs x 64 lanes x 2.4 GHz). Pair operations
(transcendental + add) report the pair. Run: python -m paper_1708_00765_amd.microbench
"""
from __future__ import annotations

import ctypes
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "microbench.hip")
LIB = os.path.join(HERE, "libcls_microbench.so")

OPS = ["fma_f32", "mad_u64_u32(+xor)", "mul_hi_u32(+add)", "log_f32(+add)", "sin_f32(+add)",
       "sqrt_f32(+add)", "rcp_f32(+add)", "fma_f64", "bitop3", "log_f64(+add)", "sincos_f64(+2add)",
       "sqrt_f64(+add)", "div_f64(+add)", "philox4x32_10 block (5 uniforms)", "lds_add_f64(+lcg)"]

PEAK_LANE_OPS = 256 * 64 * 2.4e9


def build() -> str:
    from ._build import FLAGS, HIPCC
    flags = [f for f in FLAGS if f != "-ffp-contract=off"]
    subprocess.check_call([HIPCC, *flags, SRC, "-o", LIB])
    return LIB


def run(blocks: int = 8192, iters: int = 2000) -> list[dict]:
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    lib.clsmb_run.restype = ctypes.c_double
    lib.clsmb_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    chains = lib.clsmb_chains()
    out = []
    for op, name in enumerate(OPS):
        it = iters if op not in (9, 10, 13) else max(1, iters // 20)
        ms = lib.clsmb_run(op, blocks, it)
        if ms <= 0:
            raise RuntimeError(f"microbenchmark {name} failed ({ms})")
        ops = blocks * 256.0 * it * chains
        rate = ops / (ms * 1e-3)
        out.append({"op": name, "lane_ops_per_s": rate, "frac_of_full_rate": rate / PEAK_LANE_OPS,
                    "slots_per_op": PEAK_LANE_OPS / rate})
    return out


if __name__ == "__main__":
    for r in run():
        print(json.dumps(r), flush=True)
    sys.exit(0)
