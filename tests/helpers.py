"""Shared test helpers: run a Spec through the GPU library or the oracle, compare."""
from __future__ import annotations

import numpy as np
from scipy.stats import binom

from oracle import oracle
from paper_1708_00765_amd.inputs import Spec

GEOM = {"rod": oracle.ROD, "slab": oracle.SLAB, "ext2d": oracle.EXT2D, "cube3d": oracle.CUBE3D}

# Per-bin rule: under the null each |z| > 4 with probability 6.3e-5; allow up to
# the 0.999 quantile of the binomial count over all compared bins.
P_BEYOND_4 = 6.334e-5


def oracle_problem(s: Spec) -> oracle.Problem:
    return oracle.Problem(geom=GEOM[s.geom_name], sigma=s.sigma, c=s.c, lam=s.lam, nbins=s.nbins,
                          L=s.L, source=s.source,
                          estimator=oracle.EST_COLLISION if s.collision else oracle.EST_TRACK)


def run_oracle(s: Spec, histories=None, seed=None, trace=False, threads=0):
    return oracle.run(oracle_problem(s), histories or s.histories,
                      s.seed if seed is None else seed, trace=trace, threads=threads)


def gpu_flags(s: Spec, fp32=False, trace=False):
    from paper_1708_00765_amd import cls
    f = 0
    if s.slab:
        f |= cls.CLS_F_D1_SLAB
    if s.collision:
        f |= cls.CLS_F_COLLISION_FLUX
    if fp32:
        f |= cls.CLS_F_FP32
    if trace:
        f |= cls.CLS_F_TRACE
    return f


def gpu_problem(s: Spec, fp32=False, trace=False):
    from paper_1708_00765_amd import cls
    return cls.cls_create_problem(s.d, s.L, s.sigma, s.c, s.lam, source=s.source, nbins=s.nbins,
                                  flags=gpu_flags(s, fp32, trace))


def run_gpu(s: Spec, histories=None, seed=None, fp32=False, trace_n=0):
    """Returns (tallies dict, flux, flux_sigma, trace or None)."""
    from paper_1708_00765_amd import cls
    p = gpu_problem(s, fp32=fp32, trace=trace_n > 0)
    try:
        if trace_n:
            cls.cls_set_trace_histories(p, trace_n)
        cls.cls_run(p, histories or s.histories, s.seed if seed is None else seed)
        t, flux, fsig = cls.cls_read_tallies(p, s.nbins)
        tr = cls.cls_read_trace(p, trace_n) if trace_n else None
    finally:
        cls.cls_destroy_problem(p)
    return tallies_dict(t), flux, fsig, tr


def tallies_dict(t) -> dict:
    return {k: getattr(t, k) for k, _ in t._fields_}


def z(a, sa, b, sb):
    s = np.hypot(sa, sb)
    return np.where(s > 0, (np.asarray(a) - np.asarray(b)) / np.where(s > 0, s, 1.0),
                    np.where(np.asarray(a) == np.asarray(b), 0.0, np.inf))


def allowed_beyond_4(nbins_total: int) -> int:
    return int(binom.ppf(0.999, nbins_total, P_BEYOND_4))


def compare_scalars(g: dict, o, tol=4.0):
    """GPU tallies vs oracle Result at `tol` combined sigma (independent streams)."""
    out = {}
    for key, gk, gs, ok, os_ in (("T", "T", "sigma_T", o.T, o.sigma_T),
                                 ("R", "R", "sigma_R", o.R, o.sigma_R),
                                 ("A", "A", "sigma_A", o.A, o.sigma_A),
                                 ("flux", "total_flux", "sigma_total_flux", o.total_flux,
                                  o.total_flux_sigma)):
        out[key] = float(z(g[gk], g[gs], ok, os_))
    bad = {k: v for k, v in out.items() if not abs(v) <= tol}
    return out, bad
