"""C ABI checks that need no GPU: the library loads, exports every function that
include/cls.h declares, validates arguments and reports errors by status code."""
from __future__ import annotations

import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cls.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(cls_[a-z_]+)\s*\(", text))
    return sorted(n for n in names if n not in ("cls_status",))


@pytest.fixture(scope="module")
def cls():
    from paper_1708_00765_amd import cls as mod
    return mod


def test_every_declared_function_is_exported(cls):
    names = declared_functions()
    assert len(names) >= 33
    for n in names:
        assert hasattr(cls._lib, n), n
    assert set(names) == set(cls.EXPORTED)


def test_status_strings_and_version(cls):
    assert cls.cls_status_string(cls.CLS_OK) == "CLS_OK"
    assert cls.cls_status_string(cls.CLS_ERR_EVENT_CAP) == "CLS_ERR_EVENT_CAP"
    assert cls.cls_status_string(99) == "CLS_ERR_UNKNOWN"
    assert cls.cls_version().startswith("cls-mi355x")


GOOD = dict(d=3, L=10.0, sigma_t=(0.5, 1.0), c=(0.2, 0.9), lam=(1.0, 0.3))


@pytest.mark.parametrize("bad", [
    dict(d=0), dict(d=4), dict(L=0.0), dict(L=-1.0), dict(L=math.inf), dict(L=math.nan),
    dict(sigma_t=(0.0, 1.0)), dict(sigma_t=(1.0, -2.0)), dict(sigma_t=(math.nan, 1.0)),
    dict(c=(1.01, 0.5)), dict(c=(-0.1, 0.5)), dict(c=(math.nan, 0.5)),
    dict(lam=(0.0, 1.0)), dict(lam=(math.inf, 1.0)),
    dict(source=2), dict(nbins=0), dict(nbins=8193), dict(flags=1 << 7),
    dict(flags=1),                      # slab flag with d = 3
    dict(flags=1 << 4),                 # event-only trace hash without a trace
    dict(boundaries=0),                 # vacuum lateral faces
    dict(boundaries=0b111111 | 1),      # reflecting x-face
])
def test_invalid_arguments_are_rejected(cls, bad):
    kw = dict(GOOD)
    kw.update(bad)
    with pytest.raises(cls.ClsError) as ei:
        cls.cls_create_problem(**kw)
    assert ei.value.status == cls.CLS_ERR_INVALID_ARG
    assert cls.cls_last_error()


def test_valid_problems_and_host_calls(cls):
    for d, flags, bc in ((1, 0, 0), (1, cls.CLS_F_D1_SLAB, 0), (2, cls.CLS_F_FP32, 0b1100),
                         (3, cls.CLS_F_TRACE | cls.CLS_F_COLLISION_FLUX, 0b111100),
                         (3, 0, cls.CLS_BC_DEFAULT)):
        p = cls.cls_create_problem(d, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3), nbins=2048,
                                   flags=flags, boundaries=bc)
        assert cls.cls_footprint(p, 10**6) >= 2 * 2048 * 8
        cls.cls_set_stream(p, None)
        if flags & cls.CLS_F_TRACE:
            cls.cls_set_trace_histories(p, 1000)
            assert cls.cls_footprint(p, 10**6) > cls.cls_footprint(p, 1)
        else:
            with pytest.raises(cls.ClsError):
                cls.cls_set_trace_histories(p, 10)
        # reading before any run is a state error, not a crash
        with pytest.raises(cls.ClsError) as ei:
            cls.cls_read_tallies(p, 2048)
        assert ei.value.status == cls.CLS_ERR_STATE
        with pytest.raises(cls.ClsError):
            cls.cls_run(p, 0, 1)                 # zero histories
        cls.cls_destroy_problem(p)
    cls.cls_destroy_problem(None)


def test_launch_config_validation(cls):
    old = cls.cls_get_launch_config()
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(waves_per_block=9)
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(max_chunk=10)
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(waves_per_block=3)
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(refill_min=65)
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(slots=3)
    with pytest.raises(cls.ClsError):
        cls.cls_set_launch_config(chunk_batches=2)
    cls.cls_set_launch_config(2, 4, 1024, 8, 1, 1)
    assert cls.cls_get_launch_config() == {"waves_per_block": 2, "blocks_per_cu": 4, "max_chunk": 1024,
                                           "refill_min": 8, "slots": 1, "chunk_batches": 1}
    cls.cls_set_launch_config(0, 0, 0, 0)
    assert cls.cls_get_launch_config() == old


def test_server_and_graph_need_a_device(cls):
    # without a GPU the server and graph batches fail cleanly with a status code
    with pytest.raises(cls.ClsError) as ei:
        cls.cls_server_create()
    assert ei.value.status == cls.CLS_ERR_NO_DEVICE
    p = cls.cls_create_problem(3, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3))
    try:
        with pytest.raises(cls.ClsError) as ei:
            cls.cls_batch_create([p])
        assert ei.value.status == cls.CLS_ERR_NO_DEVICE
        t = cls.cls_create_problem(3, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3), flags=cls.CLS_F_TRACE)
        with pytest.raises(cls.ClsError) as ei:      # traces are not recorded by graph batches
            cls.cls_batch_create([t])
        assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        cls.cls_destroy_problem(t)
        with pytest.raises(cls.ClsError) as ei:
            cls.cls_autotune([p], [0])
        assert ei.value.status == cls.CLS_ERR_INVALID_ARG
    finally:
        cls.cls_destroy_problem(p)


def test_batch_argument_validation(cls):
    a = cls.cls_create_problem(3, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3))
    b = cls.cls_create_problem(2, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3))
    try:
        with pytest.raises(cls.ClsError):                 # mixed geometry
            cls.cls_run_batch([a, b], [10, 10], [1, 2])
        with pytest.raises(cls.ClsError):                 # same handle twice
            cls.cls_run_batch([a, a], [10, 10], [1, 2])
        with pytest.raises(cls.ClsError):                 # zero histories
            cls.cls_run_batch([a], [0], [1])
        c = cls.cls_create_problem(3, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3))
        try:
            # argument errors come before any device work, with or without a GPU
            for call in (lambda: cls.cls_run_batch([a, c], [2**63, 2**63], [1, 2]),   # total overflows
                         lambda: cls.cls_autotune([a, c], [2**63, 2**63]),
                         lambda: cls.cls_batch_create([a, a]),
                         lambda: cls.cls_batch_create([a, b]),
                         lambda: cls.cls_autotune([c, a, c], [10, 10, 10])):
                with pytest.raises(cls.ClsError) as ei:
                    call()
                assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        finally:
            cls.cls_destroy_problem(c)
    finally:
        cls.cls_destroy_problem(a)
        cls.cls_destroy_problem(b)


def test_quenched_arguments_and_device(cls):
    slab = cls.cls_create_problem(1, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3), flags=cls.CLS_F_D1_SLAB)
    cube = cls.cls_create_problem(3, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3))
    f32 = cls.cls_create_problem(1, 10.0, (0.5, 1.0), (0.2, 0.9), (1.0, 0.3), flags=cls.CLS_F_FP32)
    fine = cls.cls_create_problem(1, 10.0, (0.5, 1.0), (0.2, 0.9), (0.005, 0.005))   # ~2000 layers expected
    try:
        for p, m, n in ((cube, 10, 10), (f32, 10, 10), (slab, 0, 10), (slab, 10, 0), (fine, 10, 10)):
            with pytest.raises(cls.ClsError) as ei:
                cls.cls_run_quenched(p, m, n, 1)
            assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        with pytest.raises(cls.ClsError) as ei:            # nothing to read yet
            cls.cls_read_quenched(slab, 100)
        assert ei.value.status == cls.CLS_ERR_STATE
        with pytest.raises(cls.ClsError) as ei:            # valid arguments, no GPU here
            cls.cls_run_quenched(slab, 10, 10, 1)
        assert ei.value.status == cls.CLS_ERR_NO_DEVICE
        assert cls.cls_status_string(cls.CLS_ERR_CAPACITY) == "CLS_ERR_CAPACITY"
    finally:
        for p in (slab, cube, f32, fine):
            cls.cls_destroy_problem(p)
