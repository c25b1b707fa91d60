"""Algorithmic work model of CLS tracking on the CDNA vector ALU (VALU).

CLS transport moves almost no data: a problem is ~10 scalars in and 2K doubles
out, and a particle's state lives in registers. The bound is the VALU issue
rate, so the roofline is counted in VALU issue slots: one slot = one wave64
lane-operation at full rate; an operation with a quarter-rate pipe
(transcendentals, 32x32 -> 64-bit integer multiply) costs 4 slots.

Peak: 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 slots/s
(equivalently the FP32 vector peak of 157.3 TFLOP/s divided by 2 for packed
issue and by 2 for the fused multiply-add).

Algorithmic slots per unit of work, counted from the operations the method
needs (Algorithm A, Section 4 of arXiv 1708.00765) and nothing else -- no
register moves, control flow, divergence or bookkeeping:

event step (every flight and every source sample), one Philox4x32-10 block:
  10 rounds x (2 x 32x32->64 multiply [4 each] + 2 three-input XOR + 2 key adds) = 120
  five 23-bit uniforms: 4 shifts + 3 bit-field ops + 5 int->float + 5 scale     =  17
flight (in addition to the step):
  material selection of 1/Sigma, Lambda, c                                       =   3
  two -ln U (log2 [4] + scale [1] each) and the two distances                    =  12
  distance to each face: subtract, scale, compare-select (4 per axis, +1 FP64)   =  4*axes + 1
  minimum of three and event code                                                =   4
  move (per axis one FMA; x in FP64) and boundary snap                           =  axes + 2
  track-length score: two bin indices (3 each), partial overlaps (6),
  four LDS addresses (4)                                                         =  16
  event dispatch and material switch                                             =   3
scatter (in addition to its flight), 3D and 2D:
  mu = 2U - 1, sin and cos of 2 pi U [4 each], sqrt(1 - mu^2) [4 + 2],
  two products, three reciprocals of the direction [4 each], 2D chord factor
  (rsqrt [4] + 3)                                                                =  28 (3D), 35 (2D)
source (in addition to its step): material choice, sqrt [4], sin/cos [8],
  sqrt(1-U) [5], lateral positions, reciprocals [12]                             =  33
lateral reflection: negate one direction component and its reciprocal          =   2
"""
from __future__ import annotations

PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9     # 3.93e13

AXES = {"rod": 1, "slab": 1, "ext2d": 2, "cube3d": 3}

STEP = 120 + 17
SOURCE = 33
LATERAL = 2


def flight_slots(geom: str) -> int:
    a = AXES[geom]
    return 3 + 12 + (4 * a + 1) + 4 + (a + 2) + 16 + 3


def scatter_slots(geom: str) -> int:
    if geom == "ext2d":
        return 35
    if geom == "cube3d":
        return 28
    return 6          # rod: a sign from one uniform; slab: mu = 2U - 1 and its reciprocal


def algorithmic_slots(geom: str, histories: int, flights: int, scatters: int, lateral: int) -> float:
    """Algorithmic VALU slots of a run from its event counters."""
    steps = histories + flights
    return (steps * STEP + flights * flight_slots(geom) + scatters * scatter_slots(geom)
            + histories * SOURCE + lateral * LATERAL)
