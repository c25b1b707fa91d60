"""ctypes front end of the FP64 CPU oracle for Chord Length Sampling.

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module. It loads
``oracle/libcls_oracle.so`` (built from ``cls_oracle.c`` with gcc) and turns the
raw sums into the paper's observables (Section 2): transmission <T> = <J_{x=L}>,
reflection <R> = <J_{x=0}>, the scalar flux on the x-mesh <phi(x)>, the total
flux <phi> = integral of <phi(x)> dx, all per source history, each with its
one-sigma statistical uncertainty computed from per-history sums.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cls_oracle.c")
LIB = os.path.join(HERE, "libcls_oracle.so")

ROD, SLAB, EXT2D, CUBE3D = 0, 1, 2, 3
SRC_FACE, SRC_VOLUME = 0, 1
EST_COLLISION, EST_TRACK = 0, 1
GEOMS = {"rod": ROD, "slab": SLAB, "ext2d": EXT2D, "cube3d": CUBE3D}

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wextra"]


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle library with gcc (always, unless force is False and it exists)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-I", HERE, src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int), ("source", ctypes.c_int), ("estimator", ctypes.c_int),
                ("nbins", ctypes.c_int), ("L", ctypes.c_double),
                ("sigma", ctypes.c_double * 2), ("c", ctypes.c_double * 2),
                ("lam", ctypes.c_double * 2), ("max_steps", ctypes.c_uint64)]


class _Counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("histories", "transmitted", "reflected", "absorbed", "capped",
                 "flights", "collisions", "scatters", "interfaces", "lateral")] + \
               [("score_sum", ctypes.c_double), ("score_sq", ctypes.c_double)]


class _Quenched(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("realizations", "histories", "transmitted", "reflected", "absorbed", "capped",
                 "flights", "collisions", "scatters", "crossings", "layers")] + \
               [("sum", ctypes.c_double * 5), ("sq", ctypes.c_double * 5)]


_lib = None


def load_library(path: str):
    """Load an oracle library from `path` (the tests also load deliberately
    mutated builds this way)."""
    lib = ctypes.CDLL(path)
    _declare(lib)
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load_library(LIB)
    return _lib


def _declare(lib):
    lib.orc_run.argtypes = [ctypes.POINTER(_Problem), ctypes.c_uint64, ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Counts),
                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_step_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_void_p]
    lib.orc_step_uniforms.restype = None
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_quenched_layers.argtypes = [ctypes.POINTER(_Problem), ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.orc_quenched_layers.restype = ctypes.c_int
    lib.orc_run_quenched.argtypes = [ctypes.POINTER(_Problem), ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.POINTER(_Quenched), ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_run_quenched.restype = ctypes.c_int


@dataclass
class Problem:
    """One CLS problem: geometry, materials (index 0 and 1), mesh and source."""
    geom: int
    sigma: tuple
    c: tuple
    lam: tuple
    nbins: int = 100
    L: float = 10.0
    source: int = SRC_FACE
    estimator: int = EST_TRACK
    max_steps: int = 0

    def _c(self) -> _Problem:
        p = _Problem()
        p.geom, p.source, p.estimator, p.nbins = int(self.geom), int(self.source), int(self.estimator), int(self.nbins)
        p.L = float(self.L)
        for i in range(2):
            p.sigma[i] = float(self.sigma[i])
            p.c[i] = float(self.c[i])
            p.lam[i] = float(self.lam[i])
        p.max_steps = int(self.max_steps)
        return p


@dataclass
class Result:
    histories: int
    transmitted: int
    reflected: int
    absorbed: int
    capped: int
    flights: int
    collisions: int
    scatters: int
    interfaces: int
    lateral: int
    T: float
    R: float
    A: float
    sigma_T: float
    sigma_R: float
    sigma_A: float
    flux: np.ndarray
    flux_sigma: np.ndarray
    total_flux: float
    total_flux_sigma: float
    bin_sum: np.ndarray
    bin_sq: np.ndarray
    score_sum: float
    score_sq: float
    trace_hash: np.ndarray | None = field(default=None)
    trace_len: np.ndarray | None = field(default=None)


def _mean_sigma(s: float, q: float, n: int) -> tuple[float, float]:
    """Mean and one-sigma error of the mean from a sum and a sum of squares of n samples."""
    if n == 0:
        return 0.0, 0.0
    mean = s / n
    if n < 2:
        return mean, 0.0
    var = max(q / n - mean * mean, 0.0) * n / (n - 1)
    return mean, float(np.sqrt(var / n))


def philox4x32_10(ctr, key, lib=None) -> tuple:
    lib = lib or _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.orc_philox4x32_10(ctypes.addressof(c), ctypes.addressof(k), ctypes.addressof(o))
    return tuple(o)


def step_uniforms(seed: int, h: int, step: int, lane: int = 0, lib=None) -> np.ndarray:
    lib = lib or _load()
    u = np.zeros(5, dtype=np.float64)
    lib.orc_step_uniforms(seed, h, step, lane, u.ctypes.data)
    return u


def max_threads() -> int:
    return int(_load().orc_max_threads())


def run(problem: Problem, histories: int, seed: int, h0: int = 0, threads: int = 0,
        trace: bool = False, lib=None) -> Result:
    """Run histories h0 .. h0+histories-1 of `problem` with stream key `seed`."""
    lib = lib or _load()
    K = int(problem.nbins)
    cnt = _Counts()
    bsum = np.zeros(K, dtype=np.float64)
    bsq = np.zeros(K, dtype=np.float64)
    th = np.zeros(histories, dtype=np.uint64) if trace else None
    tl = np.zeros(histories, dtype=np.uint32) if trace else None
    cp = problem._c()
    rc = lib.orc_run(ctypes.byref(cp), seed, h0, histories, threads, ctypes.byref(cnt),
                     bsum.ctypes.data, bsq.ctypes.data,
                     th.ctypes.data if trace else None, tl.ctypes.data if trace else None)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    N = int(cnt.histories)
    dx = problem.L / K
    T, sT = _mean_sigma(cnt.transmitted, cnt.transmitted, N)
    R, sR = _mean_sigma(cnt.reflected, cnt.reflected, N)
    A, sA = _mean_sigma(cnt.absorbed, cnt.absorbed, N)
    flux = np.zeros(K)
    fsig = np.zeros(K)
    for k in range(K):
        m, s = _mean_sigma(bsum[k], bsq[k], N)
        flux[k] = m / dx
        fsig[k] = s / dx
    tot, stot = _mean_sigma(cnt.score_sum, cnt.score_sq, N)
    return Result(histories=N, transmitted=int(cnt.transmitted), reflected=int(cnt.reflected),
                  absorbed=int(cnt.absorbed), capped=int(cnt.capped), flights=int(cnt.flights),
                  collisions=int(cnt.collisions), scatters=int(cnt.scatters),
                  interfaces=int(cnt.interfaces), lateral=int(cnt.lateral),
                  T=T, R=R, A=A, sigma_T=sT, sigma_R=sR, sigma_A=sA, flux=flux, flux_sigma=fsig,
                  total_flux=tot, total_flux_sigma=stot, bin_sum=bsum, bin_sq=bsq,
                  score_sum=float(cnt.score_sum), score_sq=float(cnt.score_sq),
                  trace_hash=th, trace_len=tl)


# ---------------------------------------------------------------------------
# Quenched disorder in d = 1 (Section 3): ensemble averages over realizations
# ---------------------------------------------------------------------------
@dataclass
class QuenchedResult:
    """Ensemble averages over realizations (Sec. 3.3) of the per-realization
    history means; each sigma is the standard error of the mean over the M
    independent realizations (it contains both the spread of the geometries
    and the transport noise of each realization)."""
    realizations: int
    histories: int
    transmitted: int
    reflected: int
    absorbed: int
    capped: int
    flights: int
    collisions: int
    scatters: int
    crossings: int
    layers: int
    T: float
    R: float
    A: float
    total_flux: float
    sigma_T: float
    sigma_R: float
    sigma_A: float
    total_flux_sigma: float
    Lk: float               # leakage <(T + R)/2> (Sec. 2, suite II)
    sigma_Lk: float
    sigma_G: tuple          # spread of the per-realization T, R, A, total flux, leakage
    flux: np.ndarray
    flux_sigma: np.ndarray
    sums: tuple
    sqs: tuple
    bin_sum: np.ndarray
    bin_sq: np.ndarray


def _ensemble(s: float, q: float, m: int) -> tuple[float, float, float]:
    """Mean, standard error of the mean and spread of m per-realization values."""
    if m == 0:
        return 0.0, 0.0, 0.0
    mean = s / m
    if m < 2:
        return mean, 0.0, 0.0
    var = max(q / m - mean * mean, 0.0) * m / (m - 1)
    return mean, float(np.sqrt(var / m)), float(np.sqrt(var))


def quenched_layers(problem: Problem, seed: int, k: int, cap: int = 1 << 16, lib=None):
    """Layers of realization k: (bounds[n+1], materials[n])."""
    lib = lib or _load()
    b = np.zeros(cap + 1, dtype=np.float64)
    m = np.zeros(cap, dtype=np.int32)
    cp = problem._c()
    n = lib.orc_quenched_layers(ctypes.byref(cp), seed, k, b.ctypes.data, m.ctypes.data, cap)
    if n < 0:
        raise ValueError("oracle rejected the problem")
    if n > cap:
        raise ValueError(f"realization has {n} layers, more than {cap}")
    return b[:n + 1].copy(), m[:n].copy()


def run_quenched(problem: Problem, realizations: int, histories: int, seed: int, k0: int = 0,
                 threads: int = 0, lib=None) -> QuenchedResult:
    """Realizations k0 .. k0+M-1 of the d = 1 Markov medium, N histories each."""
    lib = lib or _load()
    K = int(problem.nbins)
    q = _Quenched()
    bsum = np.zeros(K, dtype=np.float64)
    bsq = np.zeros(K, dtype=np.float64)
    cp = problem._c()
    rc = lib.orc_run_quenched(ctypes.byref(cp), seed, k0, realizations, histories, threads,
                              ctypes.byref(q), bsum.ctypes.data, bsq.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the quenched problem")
    M = int(q.realizations)
    obs = [_ensemble(q.sum[j], q.sq[j], M) for j in range(5)]
    dx = problem.L / K
    flux = np.zeros(K)
    fsig = np.zeros(K)
    for b in range(K):
        mean, sig, _ = _ensemble(bsum[b], bsq[b], M)
        flux[b] = mean / dx
        fsig[b] = sig / dx
    return QuenchedResult(
        realizations=M, histories=int(q.histories), transmitted=int(q.transmitted),
        reflected=int(q.reflected), absorbed=int(q.absorbed), capped=int(q.capped),
        flights=int(q.flights), collisions=int(q.collisions), scatters=int(q.scatters),
        crossings=int(q.crossings), layers=int(q.layers),
        T=obs[0][0], R=obs[1][0], A=obs[2][0], total_flux=obs[3][0],
        sigma_T=obs[0][1], sigma_R=obs[1][1], sigma_A=obs[2][1], total_flux_sigma=obs[3][1],
        Lk=obs[4][0], sigma_Lk=obs[4][1],
        sigma_G=tuple(o[2] for o in obs), flux=flux, flux_sigma=fsig,
        sums=tuple(q.sum), sqs=tuple(q.sq), bin_sum=bsum, bin_sq=bsq)
