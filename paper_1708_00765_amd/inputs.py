"""Seeded synthetic workloads for the CLS library and its tests.

This module only draws problem parameters and run seeds; it holds none of the
transport arithmetic, so both the GPU path and the CPU oracle can be fed from it.

Workloads (parameter laws per benchmark configuration; L = 10 everywhere, the box
of Section 2 of Larmier et al., arXiv 1708.00765):
  rod_collision   d=1 rod, 1 set, 1e5 histories, 100 bins, collision estimator.
  cube3d_track    d=3 cube, 8 sets, 1e8 histories per set, 200 bins, track length.
  ext2d_batched   d=2 extruded, 256 sets, histories log-uniform in [1e4, 1e7],
                  bins uniform in [100, 1000], track length.
  served          requests with d uniform in {1, 2, 3}, histories log-uniform in
                  [1e4, 1e8], bins uniform in [10, 1000], Poisson arrivals.
  stress3d        d=3 cube, 32 sets, c in [0.99, 0.999], Sigma in [0.5, 5],
                  Lambda in [0.05, 1], 1e8 histories per set, 1000 bins.
Common law (first four): Sigma_i log-uniform in [0.02, 2], c_i uniform in [0, 1],
Lambda_i log-uniform in [0.1, 10].
The paper's own benchmark (Tables 1 and 2) is `paper_cases()`.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

L_BOX = 10.0
PARAM_SEED_BASE = 20170802
RUN_SEED_BASE = 765

WORKLOADS = ("rod_collision", "cube3d_track", "ext2d_batched", "served", "stress3d")


@dataclass
class Spec:
    """One CLS problem and its run: everything both sides need."""
    d: int
    sigma: tuple
    c: tuple
    lam: tuple
    nbins: int
    histories: int
    seed: int
    L: float = L_BOX
    slab: bool = False
    source: int = 0           # 0 = incident flux on x=0, 1 = interior source
    collision: bool = False   # collision estimator (else track length)
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def geom_name(self) -> str:
        if self.d == 1:
            return "slab" if self.slab else "rod"
        return "ext2d" if self.d == 2 else "cube3d"


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (seed derivation only)."""
    z = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def run_seed(workload_index: int, j: int, salt: int = 0) -> int:
    return splitmix64(RUN_SEED_BASE + workload_index + 1000003 * salt + 7919 * j)


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _common_law(rng):
    sig = _loguniform(rng, 0.02, 2.0, 2)
    c = rng.uniform(0.0, 1.0, 2)
    lam = _loguniform(rng, 0.1, 10.0, 2)
    return tuple(map(float, sig)), tuple(map(float, c)), tuple(map(float, lam))


def workload(name: str, histories: int | None = None, salt: int = 0) -> list[Spec]:
    """Parameter sets of a workload. `histories` overrides the per-set history
    count (smaller parity runs); `salt` changes the run seeds only."""
    idx = WORKLOADS.index(name)
    rng = np.random.default_rng(PARAM_SEED_BASE + idx)
    out: list[Spec] = []
    if name == "rod_collision":
        s, c, l = _common_law(rng)
        out.append(Spec(1, s, c, l, 100, histories or 100_000, run_seed(idx, 0, salt),
                        collision=True, name="rod_collision[0]"))
    elif name == "cube3d_track":
        for j in range(8):
            s, c, l = _common_law(rng)
            out.append(Spec(3, s, c, l, 200, histories or 100_000_000, run_seed(idx, j, salt),
                            name=f"cube3d_track[{j}]"))
    elif name == "ext2d_batched":
        for j in range(256):
            s, c, l = _common_law(rng)
            n = int(round(float(_loguniform(rng, 1e4, 1e7))))
            k = int(rng.integers(100, 1001))
            out.append(Spec(2, s, c, l, k, histories or n, run_seed(idx, j, salt),
                            name=f"ext2d_batched[{j}]"))
    elif name == "stress3d":
        for j in range(32):
            sig = tuple(map(float, _loguniform(rng, 0.5, 5.0, 2)))
            c = tuple(map(float, rng.uniform(0.99, 0.999, 2)))
            lam = tuple(map(float, _loguniform(rng, 0.05, 1.0, 2)))
            out.append(Spec(3, sig, c, lam, 1000, histories or 100_000_000, run_seed(idx, j, salt),
                            name=f"stress3d[{j}]"))
    elif name == "served":
        raise ValueError("use served_requests() for the request stream")
    else:
        raise KeyError(name)
    return out


def served_requests(rate_hz: float = 200.0, duration_s: float = 60.0, salt: int = 0,
                    max_histories: float = 1e8):
    """Poisson request stream: list of (arrival_time_s, Spec)."""
    idx = WORKLOADS.index("served")
    rng = np.random.default_rng(PARAM_SEED_BASE + idx + 1000 * salt)
    t = 0.0
    reqs = []
    j = 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        d = int(rng.integers(1, 4))
        s, c, l = _common_law(rng)
        n = int(round(float(_loguniform(rng, 1e4, max_histories))))
        k = int(rng.integers(10, 1001))
        reqs.append((t, Spec(d, s, c, l, k, n, run_seed(idx, j, salt), collision=(d == 1),
                             name=f"served[{j}]")))
        j += 1
    return reqs


# The paper's benchmark materials (Table 1) and scattering ratios (Table 2).
PAPER_MATERIALS = {
    "1": (Fraction(10, 99), Fraction(99, 100), Fraction(100, 11), Fraction(11, 100)),
    "2": (Fraction(10, 99), Fraction(99, 10), Fraction(100, 11), Fraction(11, 10)),
    "3": (Fraction(2, 101), Fraction(101, 20), Fraction(200, 101), Fraction(101, 20)),
}
PAPER_SCATTERING = {"a": (0.0, 1.0), "b": (1.0, 0.0), "c": (0.9, 0.9)}


def paper_case(case: str, d: int, suite: str = "I", histories: int = 1_000_000, seed: int = 1,
               nbins: int = 100) -> Spec:
    """Benchmark case like '2b' in dimension d (1 = slab) for suite I or II."""
    sa, la, sb, lb = PAPER_MATERIALS[case[0]]
    c = PAPER_SCATTERING[case[1]]
    return Spec(d, (float(sa), float(sb)), c, (float(la), float(lb)), nbins, histories, seed,
                slab=(d == 1), source=0 if suite == "I" else 1, name=f"{suite}-{case}-d{d}")


def paper_cases():
    return [c + s for c in "123" for s in "abc"]
