"""Host checks of the algorithmic work model behind the bench roofline."""
from __future__ import annotations

import pytest

from paper_1708_00765_amd import perf_model as pm


@pytest.mark.parametrize("geom", ["rod", "slab", "ext2d", "cube3d"])
def test_slots_are_linear_in_the_event_counts(geom):
    a = pm.algorithmic_slots(geom, 1000, 20000, 3000, 500)
    b = pm.algorithmic_slots(geom, 2000, 40000, 6000, 1000)
    assert a > 0 and abs(b / a - 2.0) < 1e-12


def test_fp64_prices_exceed_fp32():
    t32, t64 = pm.per_unit_table(True), pm.per_unit_table(False)
    for g in t32:
        for k in ("flight", "scatter"):
            assert t64[g][k] >= t32[g][k], (g, k)
    # a FP64 flight holds two library logs
    assert t64["cube3d"]["flight"] > 2 * pm.LOG64


def test_quenched_model():
    n = 10**6
    base = pm.quenched_slots(True, True, True, n, 20 * n, 2 * n, n)
    assert abs(pm.quenched_slots(True, True, True, 2 * n, 40 * n, 4 * n, 2 * n) / base - 2.0) < 1e-12
    # one FP64 log and three divisions per flight, one Philox block per step
    per_flight = (pm.quenched_slots(True, True, True, n, 21 * n, 2 * n, n) - base) / n
    assert per_flight > pm.PHILOX + pm.LOG64 + 3 * pm.DIV64
    # the collision estimator scores at collisions, the track-length one every flight
    assert pm.quenched_slots(True, False, True, n, 20 * n, 2 * n, n) < base
