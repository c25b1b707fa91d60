"""Algorithmic work model of CLS tracking on the CDNA vector ALU (VALU).

CLS transport moves almost no data: a problem is ~10 scalars in and 2K doubles
out, and a particle's state lives in registers. The bound is VALU issue, so the
roofline is counted in VALU issue slots.

Peak (published): the FP32 vector rate of 157.3 TFLOP/s is 78.6e12 fused
multiply-adds per second, i.e. 256 compute units x 128 lanes x 2.4 GHz. One
slot = one lane-operation at that rate.

Price of each operation class, in slots = peak / (its measured throughput),
from the instruction-rate microbenchmarks (csrc/microbench.hip, results in
profiles/microbench_gfx950.md): FP32 add/mul/fma 1.36; other 32-bit VALU
operations (integer, compare, select, conversion, bit logic) 2.22; FP64
add/mul/fma 2.41; FP32 transcendental (log2, sin, cos, sqrt, rcp, rsq) 4.5;
one Philox4x32-10 block including the five 23-bit fields 88.6; FP64 log 188.5,
sincos 125, sqrt 42.2, division/reciprocal 28.4.

Operation counts per unit of work are those the method needs (Algorithm A,
Section 4 of arXiv 1708.00765), not those a particular kernel executes: no
register moves, control flow, divergence or bookkeeping. The tally additions
go to the LDS pipe and are not VALU work. With these prices an ideal kernel
that issued only the algorithm's operations back to back would reach 100%.
"""
from __future__ import annotations

PEAK_SLOTS_PER_S = 256 * 128 * 2.4e9        # 7.86e13 (= 157.3 TFLOP/s / 2)

# measured prices (slots per lane-operation)
F32, I32, F64, TR32 = 1.36, 2.22, 2.41, 4.5
PHILOX = 88.6
LOG64, SINCOS64, SQRT64, DIV64 = 188.5, 125.0, 42.2, 28.4

AXES = {"rod": 1, "slab": 1, "ext2d": 2, "cube3d": 3}


def _price(fp32: bool, f32=0, i32=0, f64=0, tr=0, log=0, sincos=0, sqrt=0, rcp=0):
    """Slots of an operation mix; `log`, `sincos`, `sqrt`, `rcp` are the
    precision-dependent calls (FP32 hardware, FP64 library)."""
    if fp32:
        return f32 * F32 + i32 * I32 + f64 * F64 + (tr + log + 2 * sincos + sqrt + rcp) * TR32
    return (f32 * F64 + i32 * I32 + f64 * F64 + tr * TR32 + log * LOG64 + sincos * SINCOS64
            + sqrt * SQRT64 + rcp * DIV64)


def step_slots(fp32: bool) -> float:
    """Every event step (source or flight): one Philox block, five uniforms."""
    return PHILOX + _price(fp32, i32=5, f32=5)


def flight_slots(geom: str, fp32: bool, track: bool = True) -> float:
    lat = AXES[geom] - 1
    ops = dict(
        i32=3                              # material selection of 1/Sigma, Lambda, c
        + 2 + 3 * lat                      # boundary: x face select, per lateral axis compare + 2 selects
        + 5                                # minimum of three and event code
        + 1 + 2                            # move: x conversion, boundary snap
        + 3                                # bin index of the new position
        + (2 + 1 + 2 + 4 if track else 1)  # track score: ordering, same-bin test, edges, 4 LDS addresses
        + 3,                               # event dispatch and material switch
        f32=5                              # distance scalings
        + 1 + 2 * lat                      # boundary: x scale, per lateral axis subtract + scale
        + 1 + lat,                         # move: s*ux, lateral FMAs
        f64=1 + 1 + 1 + (10 if track else 0),   # x distance, x move, bin scale, track partials
        log=2,
    )
    return _price(fp32, **ops)


def scatter_slots(geom: str, fp32: bool) -> float:
    if geom == "rod":
        return _price(fp32, i32=2)
    if geom == "slab":
        return _price(fp32, f32=2, rcp=1)
    extra = dict(tr=1, f32=3) if geom == "ext2d" else {}
    ops = dict(f32=1 + 3 + 2 + extra.get("f32", 0), sincos=1, sqrt=1, rcp=3, tr=extra.get("tr", 0))
    return _price(fp32, **ops)


def source_slots(geom: str, fp32: bool) -> float:
    base = _price(fp32, i32=2 + 3, f64=1)          # material, bin of the entry point
    if geom == "rod":
        return base
    if geom == "slab":
        return base + _price(fp32, sqrt=1, rcp=1)
    return base + scatter_slots(geom, fp32) + _price(fp32, f32=2)   # cosine-law direction + lateral entry


def algorithmic_slots(geom: str, histories: int, flights: int, scatters: int, lateral: int,
                      fp32: bool = True, track: bool = True) -> float:
    """Algorithmic VALU slots of a run from its event counters."""
    steps = histories + flights
    return (steps * step_slots(fp32) + flights * flight_slots(geom, fp32, track)
            + scatters * scatter_slots(geom, fp32) + histories * source_slots(geom, fp32)
            + lateral * 2 * F32)


def quenched_slots(slab: bool, track: bool, face_source: bool, histories: int, flights: int, collisions: int,
                   scatters: int) -> float:
    """Algorithmic VALU slots of a quenched-disorder run in d = 1 (Section 3),
    FP64 throughout: the realization's layers fix every interface, so a flight
    samples only the collision distance and compares it with the distance to
    the face of its layer. Building the layers (about rho L cells per
    realization, against N x flights of transport) is left out."""
    step = PHILOX + _price(False, i32=5, f64=2)                  # block, uniforms to FP64
    flight = (_price(False, log=1, rcp=3)                          # -ln u / Sigma, (face - x) / mu, 1 / |mu|
              + _price(False, i32=2 + 1 + 1 + 4 + 2,               # material, face select, compare, leak/layer tests
                       f64=1 + 1))                                 # face - x, move
    if track:
        flight += _price(False, i32=2 * 3 + 2 + 4, f64=2 + 6 + 1)   # 2 bins, ordering, 4 LDS addresses; partials
    coll = _price(False, f64=1) + (0.0 if track else _price(False, rcp=1, i32=3, f64=2))
    scatter = _price(False, f64=2) if slab else _price(False, i32=2)
    if face_source:
        source = _price(False, sqrt=1) if slab else 0.0
    else:
        source = _price(False, f64=3, i32=6 * 3)                  # x, mu, layer by bisection
    return ((histories + flights) * step + flights * flight + collisions * coll + scatters * scatter
            + histories * source)


def per_unit_table(fp32: bool = True) -> dict:
    """Slots per unit of work, for the design notes."""
    return {g: {"step": step_slots(fp32), "flight": flight_slots(g, fp32), "scatter": scatter_slots(g, fp32),
                "source": source_slots(g, fp32)} for g in AXES}
