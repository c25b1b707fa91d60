"""Thin ctypes binding of the CLS C ABI (include/cls.h), same names as the C calls.

Argument marshalling only: every step of a run executes in libcls_hip.so (HIP
kernels for gfx950). There is no fallback: if the library is not built this
module raises at import time, and a missing or non-gfx950 device surfaces as a
ClsError from the first run. PyTorch, when the caller uses it, only supplies
device memory (cls_bind_device_memory) and streams (cls_set_stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY_PATH = os.path.join(_HERE, "libcls_hip.so")

if not os.path.exists(LIBRARY_PATH):
    raise ImportError(
        f"{LIBRARY_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIBRARY_PATH)

# ---- constants (mirror include/cls.h) --------------------------------------
CLS_OK = 0
CLS_ERR_INVALID_ARG = 1
CLS_ERR_OUT_OF_MEMORY = 2
CLS_ERR_DEVICE = 3
CLS_ERR_NOT_READY = 4
CLS_ERR_EVENT_CAP = 5
CLS_ERR_STATE = 6
CLS_ERR_NO_DEVICE = 7
CLS_ERR_CAPACITY = 8

CLS_SRC_FACE_X0 = 0
CLS_SRC_VOLUME = 1
CLS_BC_DEFAULT = 0xFFFFFFFF

CLS_F_D1_SLAB = 1 << 0
CLS_F_COLLISION_FLUX = 1 << 1
CLS_F_FP32 = 1 << 2
CLS_F_TRACE = 1 << 3
CLS_F_TRACE_NO_BINS = 1 << 4

CLS_MAX_BINS = 8192

EXPORTED = (
    "cls_create_problem", "cls_destroy_problem", "cls_set_stream", "cls_footprint",
    "cls_bind_device_memory", "cls_set_trace_histories", "cls_run", "cls_run_async",
    "cls_query", "cls_synchronize", "cls_read_tallies", "cls_read_trace", "cls_run_batch",
    "cls_batch_create", "cls_batch_run", "cls_batch_last_ms", "cls_batch_destroy",
    "cls_set_launch_config", "cls_get_launch_config", "cls_autotune",
    "cls_server_create", "cls_server_submit", "cls_server_poll", "cls_server_wait",
    "cls_server_request_info", "cls_server_release", "cls_server_get_stats", "cls_server_destroy",
    "cls_run_quenched", "cls_read_quenched", "cls_run_static",
    "cls_status_string", "cls_last_error", "cls_version",
)


class cls_tallies(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "histories", "transmitted", "reflected", "absorbed", "capped", "flights", "collisions",
        "scatters", "interface_crossings", "lateral_reflections", "batches")] + \
        [(n, ctypes.c_double) for n in (
            "T", "R", "A", "sigma_T", "sigma_R", "sigma_A", "total_flux", "sigma_total_flux",
            "track_ms")]


class cls_quenched_tallies(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "realizations", "histories", "transmitted", "reflected", "absorbed", "capped", "flights",
        "collisions", "scatters", "crossings", "layers")] + \
        [(n, ctypes.c_double) for n in (
            "T", "R", "A", "total_flux", "Lk",
            "sigma_T", "sigma_R", "sigma_A", "sigma_total_flux", "sigma_Lk",
            "spread_T", "spread_R", "spread_A", "spread_total_flux", "spread_Lk", "track_ms")]


class cls_launch_config(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("max_chunk", ctypes.c_int), ("refill_min", ctypes.c_int), ("slots", ctypes.c_int),
                ("chunk_batches", ctypes.c_int)]


class cls_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("round_histories", ctypes.c_uint64),
                ("max_inflight_rounds", ctypes.c_int), ("record_path", ctypes.c_int)]


class cls_request_info(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("histories", ctypes.c_uint64), ("rounds", ctypes.c_uint32), ("publish_s", ctypes.c_double),
                ("signal_s", ctypes.c_double), ("finalize_s", ctypes.c_double)]


class cls_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "failed", "pending", "active",
                                               "rounds", "histories_completed")] + \
        [(n, ctypes.c_size_t) for n in ("hbm_in_use", "hbm_peak", "hbm_budget")] + \
        [("worker_status", ctypes.c_int), ("wave_idle_share", ctypes.c_double)]


_P = ctypes.c_void_p
_D2 = ctypes.c_double * 2


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("cls_create_problem", ctypes.c_int, ctypes.c_int, ctypes.c_double, _D2, _D2, _D2, ctypes.c_int,
     ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_P))
_sig("cls_destroy_problem", None, _P)
_sig("cls_set_stream", ctypes.c_int, _P, _P)
_sig("cls_footprint", ctypes.c_int, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_size_t))
_sig("cls_bind_device_memory", ctypes.c_int, _P, _P, ctypes.c_size_t)
_sig("cls_set_trace_histories", ctypes.c_int, _P, ctypes.c_uint64)
_sig("cls_run", ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_uint64)
_sig("cls_run_async", ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_uint64)
_sig("cls_query", ctypes.c_int, _P)
_sig("cls_synchronize", ctypes.c_int, _P)
_sig("cls_read_tallies", ctypes.c_int, _P, ctypes.POINTER(cls_tallies), _P, _P, ctypes.c_int)
_sig("cls_read_trace", ctypes.c_int, _P, _P, _P, ctypes.c_uint64)
_sig("cls_run_batch", ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64),
     ctypes.POINTER(ctypes.c_uint64), ctypes.c_int)
_sig("cls_batch_create", ctypes.c_int, ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P))
_sig("cls_batch_run", ctypes.c_int, _P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64))
_sig("cls_batch_last_ms", ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double))
_sig("cls_batch_destroy", None, _P)
_sig("cls_autotune", ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint64), ctypes.c_int,
     ctypes.c_uint64, ctypes.POINTER(cls_launch_config), ctypes.POINTER(ctypes.c_double))
_sig("cls_server_create", ctypes.c_int, ctypes.POINTER(cls_server_config), ctypes.POINTER(_P))
_sig("cls_server_submit", ctypes.c_int, _P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64))
_sig("cls_server_poll", ctypes.c_int, _P, ctypes.c_uint64)
_sig("cls_server_wait", ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_double)
_sig("cls_server_request_info", ctypes.c_int, _P, ctypes.c_uint64, ctypes.POINTER(cls_request_info))
_sig("cls_server_release", ctypes.c_int, _P, ctypes.c_uint64)
_sig("cls_server_get_stats", ctypes.c_int, _P, ctypes.POINTER(cls_server_stats))
_sig("cls_server_destroy", None, _P)
_sig("cls_set_launch_config", ctypes.c_int, ctypes.POINTER(cls_launch_config))
_sig("cls_get_launch_config", ctypes.c_int, ctypes.POINTER(cls_launch_config))
_sig("cls_run_quenched", ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64)
_sig("cls_run_static", ctypes.c_int, _P, ctypes.c_uint64, ctypes.c_uint64, _P, _P, ctypes.c_size_t)
_sig("cls_read_quenched", ctypes.c_int, _P, ctypes.POINTER(cls_quenched_tallies), _P, _P, ctypes.c_int)
_sig("cls_status_string", ctypes.c_char_p, ctypes.c_int)
_sig("cls_last_error", ctypes.c_char_p)
_sig("cls_version", ctypes.c_char_p)


class ClsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.cls_last_error().decode(errors="replace")
        name = _lib.cls_status_string(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


def _check(status: int, where: str, allow=()):
    if status != CLS_OK and status not in allow:
        raise ClsError(status, where)
    return status


# ---- the C calls ------------------------------------------------------------
def cls_create_problem(d, L, sigma_t, c, lam, source=CLS_SRC_FACE_X0, boundaries=CLS_BC_DEFAULT,
                       nbins=100, flags=0) -> int:
    """Returns the opaque problem handle (an int)."""
    h = _P()
    _check(_lib.cls_create_problem(int(d), float(L), _D2(*map(float, sigma_t)), _D2(*map(float, c)),
                                   _D2(*map(float, lam)), int(source), int(boundaries) & 0xFFFFFFFF,
                                   int(nbins), int(flags), ctypes.byref(h)), "cls_create_problem")
    return h.value


def cls_destroy_problem(p: int) -> None:
    _lib.cls_destroy_problem(p)


def cls_set_stream(p: int, hip_stream: int) -> None:
    _check(_lib.cls_set_stream(p, hip_stream), "cls_set_stream")


def cls_footprint(p: int, histories: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.cls_footprint(p, int(histories), ctypes.byref(b)), "cls_footprint")
    return b.value


def cls_bind_device_memory(p: int, dev_ptr: int, nbytes: int) -> None:
    _check(_lib.cls_bind_device_memory(p, dev_ptr, int(nbytes)), "cls_bind_device_memory")


def cls_set_trace_histories(p: int, n: int) -> None:
    _check(_lib.cls_set_trace_histories(p, int(n)), "cls_set_trace_histories")


def cls_run(p: int, histories: int, seed: int, allow_cap: bool = False) -> int:
    allow = (CLS_ERR_EVENT_CAP,) if allow_cap else ()
    return _check(_lib.cls_run(p, int(histories), int(seed) & (2**64 - 1)), "cls_run", allow)


def cls_run_async(p: int, histories: int, seed: int) -> None:
    _check(_lib.cls_run_async(p, int(histories), int(seed) & (2**64 - 1)), "cls_run_async")


def cls_query(p: int) -> bool:
    """True when the last run has completed."""
    st = _lib.cls_query(p)
    if st == CLS_ERR_NOT_READY:
        return False
    _check(st, "cls_query")
    return True


def cls_synchronize(p: int) -> None:
    _check(_lib.cls_synchronize(p), "cls_synchronize")


def cls_read_tallies(p: int, nbins: int, allow_cap: bool = False):
    """Returns (cls_tallies, flux[nbins], flux_sigma[nbins])."""
    t = cls_tallies()
    flux = np.zeros(nbins, dtype=np.float64)
    fsig = np.zeros(nbins, dtype=np.float64)
    allow = (CLS_ERR_EVENT_CAP,) if allow_cap else ()
    _check(_lib.cls_read_tallies(p, ctypes.byref(t), flux.ctypes.data, fsig.ctypes.data, int(nbins)),
           "cls_read_tallies", allow)
    return t, flux, fsig


def cls_read_trace(p: int, n: int):
    """Returns (hash[n] uint64, flights[n] uint32)."""
    hsh = np.zeros(n, dtype=np.uint64)
    fl = np.zeros(n, dtype=np.uint32)
    _check(_lib.cls_read_trace(p, hsh.ctypes.data, fl.ctypes.data, int(n)), "cls_read_trace")
    return hsh, fl


def cls_run_batch(problems, histories, seeds, allow_cap: bool = False) -> int:
    n = len(problems)
    arr = (_P * n)(*problems)
    hs = (ctypes.c_uint64 * n)(*[int(v) for v in histories])
    ss = (ctypes.c_uint64 * n)(*[int(v) & (2**64 - 1) for v in seeds])
    allow = (CLS_ERR_EVENT_CAP,) if allow_cap else ()
    return _check(_lib.cls_run_batch(arr, hs, ss, n), "cls_run_batch", allow)


def cls_set_launch_config(waves_per_block=0, blocks_per_cu=0, max_chunk=0, refill_min=0, slots=0,
                          chunk_batches=0) -> None:
    cfg = cls_launch_config(int(waves_per_block), int(blocks_per_cu), int(max_chunk), int(refill_min), int(slots),
                            int(chunk_batches))
    _check(_lib.cls_set_launch_config(ctypes.byref(cfg)), "cls_set_launch_config")


def _cfg_dict(cfg) -> dict:
    return {"waves_per_block": cfg.waves_per_block, "blocks_per_cu": cfg.blocks_per_cu,
            "max_chunk": cfg.max_chunk, "refill_min": cfg.refill_min, "slots": cfg.slots,
            "chunk_batches": cfg.chunk_batches}


def cls_get_launch_config() -> dict:
    cfg = cls_launch_config()
    _check(_lib.cls_get_launch_config(ctypes.byref(cfg)), "cls_get_launch_config")
    return _cfg_dict(cfg)


def cls_autotune(problems, histories, sample_histories: int = 0):
    """Returns (launch config dict, histories/s of the winner or 0.0 from the cache)."""
    n = len(problems)
    arr = (_P * n)(*problems)
    hs = (ctypes.c_uint64 * n)(*[int(v) for v in histories])
    cfg = cls_launch_config()
    rate = ctypes.c_double()
    _check(_lib.cls_autotune(arr, hs, n, int(sample_histories), ctypes.byref(cfg), ctypes.byref(rate)),
           "cls_autotune")
    return _cfg_dict(cfg), rate.value


# ---- graph-captured batches ---------------------------------------------------
def cls_batch_create(problems) -> int:
    n = len(problems)
    arr = (_P * n)(*problems)
    h = _P()
    _check(_lib.cls_batch_create(arr, n, ctypes.byref(h)), "cls_batch_create")
    return h.value


def cls_batch_run(b: int, histories, seeds, allow_cap: bool = False) -> int:
    n = len(histories)
    hs = (ctypes.c_uint64 * n)(*[int(v) for v in histories])
    ss = (ctypes.c_uint64 * n)(*[int(v) & (2**64 - 1) for v in seeds])
    allow = (CLS_ERR_EVENT_CAP,) if allow_cap else ()
    return _check(_lib.cls_batch_run(b, hs, ss), "cls_batch_run", allow)


def cls_batch_last_ms(b: int) -> float:
    ms = ctypes.c_double()
    _check(_lib.cls_batch_last_ms(b, ctypes.byref(ms)), "cls_batch_last_ms")
    return ms.value


def cls_batch_destroy(b: int) -> None:
    _lib.cls_batch_destroy(b)


# ---- serving -----------------------------------------------------------------
def cls_server_create(hbm_budget_bytes: int = 0, round_histories: int = 0, max_inflight_rounds: int = 0,
                      record_path: int = 0) -> int:
    cfg = cls_server_config(int(hbm_budget_bytes), int(round_histories), int(max_inflight_rounds), int(record_path))
    h = _P()
    _check(_lib.cls_server_create(ctypes.byref(cfg), ctypes.byref(h)), "cls_server_create")
    return h.value


def cls_server_submit(s: int, p: int, histories: int, seed: int) -> int:
    t = ctypes.c_uint64()
    _check(_lib.cls_server_submit(s, p, int(histories), int(seed) & (2**64 - 1), ctypes.byref(t)),
           "cls_server_submit")
    return t.value


def cls_server_poll(s: int, ticket: int) -> bool:
    st = _lib.cls_server_poll(s, int(ticket))
    if st == CLS_ERR_NOT_READY:
        return False
    _check(st, "cls_server_poll")
    return True


def cls_server_wait(s: int, ticket: int, timeout_s: float = 0.0) -> bool:
    st = _lib.cls_server_wait(s, int(ticket), float(timeout_s))
    if st == CLS_ERR_NOT_READY:
        return False
    _check(st, "cls_server_wait")
    return True


def cls_server_request_info(s: int, ticket: int) -> dict:
    info = cls_request_info()
    _check(_lib.cls_server_request_info(s, int(ticket), ctypes.byref(info)), "cls_server_request_info")
    return {k: getattr(info, k) for k, _ in info._fields_}


def cls_server_release(s: int, ticket: int) -> None:
    _check(_lib.cls_server_release(s, int(ticket)), "cls_server_release")


def cls_server_get_stats(s: int) -> dict:
    st = cls_server_stats()
    _check(_lib.cls_server_get_stats(s, ctypes.byref(st)), "cls_server_get_stats")
    return {k: getattr(st, k) for k, _ in st._fields_}


def cls_server_destroy(s: int) -> None:
    _lib.cls_server_destroy(s)


def cls_run_static(p: int, histories: int, seed: int, stream: int | None, d_record: int, record_bytes: int) -> None:
    """Allocation-free run (enqueued on `stream`; the caller synchronizes). `d_record`
    is caller-owned device memory of at least record_bytes(nbins) bytes."""
    _check(_lib.cls_run_static(p, int(histories), int(seed) & (2**64 - 1), stream or None, int(d_record),
                               int(record_bytes)), "cls_run_static")


RECORD_COUNTERS = ("histories", "transmitted", "reflected", "absorbed", "capped", "flights", "collisions",
                   "scatters", "interface_crossings", "lateral_reflections", "batches")
RECORD_DOUBLES = ("T", "R", "A", "sigma_T", "sigma_R", "sigma_A", "total_flux", "sigma_total_flux")


def record_bytes(nbins: int) -> int:
    """Size of the result record of cls_run_static: 16 counters, 8 doubles, 2 x nbins doubles."""
    return (24 + 2 * int(nbins)) * 8


def decode_record(words, nbins: int):
    """Split a result record (the 8-byte words as a numpy uint64 array) into a dict of
    the counters and scalars, flux[nbins] and flux_sigma[nbins]."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    d = w[16:].view(np.float64)
    out = {k: int(w[i]) for i, k in enumerate(RECORD_COUNTERS)}
    out.update({k: float(d[i]) for i, k in enumerate(RECORD_DOUBLES)})
    return out, d[8:8 + nbins].copy(), d[8 + nbins:8 + 2 * nbins].copy()


def cls_run_quenched(p: int, realizations: int, histories: int, seed: int) -> None:
    """Quenched-disorder reference solution of a d = 1 problem (synchronous)."""
    _check(_lib.cls_run_quenched(p, int(realizations), int(histories), int(seed) & (2**64 - 1)),
           "cls_run_quenched")


def cls_read_quenched(p: int, nbins: int):
    """Returns (cls_quenched_tallies, flux[nbins], flux_sigma[nbins])."""
    t = cls_quenched_tallies()
    flux = np.zeros(nbins, dtype=np.float64)
    fsig = np.zeros(nbins, dtype=np.float64)
    _check(_lib.cls_read_quenched(p, ctypes.byref(t), flux.ctypes.data, fsig.ctypes.data, int(nbins)),
           "cls_read_quenched")
    return t, flux, fsig


def cls_status_string(status: int) -> str:
    return _lib.cls_status_string(int(status)).decode()


def cls_last_error() -> str:
    return _lib.cls_last_error().decode(errors="replace")


def cls_version() -> str:
    return _lib.cls_version().decode()
