"""Served requests against the FP64 CPU oracle (Algorithm A, Section 4; combined
variance of Section 5).

A mixed stream of rod, extruded-2D and cube requests (10 to 1000 bins, FP64 and FP32)
goes through the continuous-batching server, whose rounds run one kernel per precision
for every kind of problem. The launch shape is narrowed (256 waves, chunks of at most
256 histories) so that the large requests run for many chunks next to the small ones.
  - FP64 requests follow the oracle's random streams: the counts equal the oracle's
    and the flux agrees to 1e-9 (summation order only);
  - FP32 requests agree with oracle runs on independent seeds within 4 combined sigma
    (T, R, A, total flux) and by the binomial per-bin 4-sigma rule;
  - the records written straight into pinned host memory equal those written to
    device memory and copied (record_path = 1) for the same requests, errors
    (sigma_*, flux_sigma) included.
All GPU calls go through the C ABI."""
from __future__ import annotations

import time

import numpy as np
import pytest

from helpers import allowed_beyond_4, gpu_problem, run_oracle, tallies_dict, z
from paper_1708_00765_amd.inputs import Spec

pytestmark = pytest.mark.gpu

COUNTS = ("histories", "transmitted", "reflected", "absorbed", "flights", "collisions", "scatters",
          "interface_crossings", "lateral_reflections", "batches")


@pytest.fixture(scope="module")
def cls():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1708_00765_amd import cls as mod
    yield mod
    mod.cls_set_launch_config(0, 0, 0, 0)


def _law(rng):
    sig = tuple(float(v) for v in np.exp(rng.uniform(np.log(0.02), np.log(2.0), 2)))
    c = tuple(float(v) for v in rng.uniform(0.0, 1.0, 2))
    lam = tuple(float(v) for v in np.exp(rng.uniform(np.log(0.1), np.log(10.0), 2)))
    return sig, c, lam


def served_mix(seed):
    """(spec, fp32) pairs: per precision a large cube (1000 bins), a large extruded
    problem and a rod (collision estimator), then small requests of every d."""
    rng = np.random.default_rng(seed)
    out = []
    for fp32 in (False, True):
        big = [(3, 1000, 2_000_000), (2, 400, 1_500_000), (1, 60, 400_000)]
        small = [(int(rng.integers(1, 4)), int(rng.integers(10, 1001)), int(10 ** rng.uniform(3.5, 5)))
                 for _ in range(6)]
        for j, (d, k, n) in enumerate(big + small):
            sig, c, lam = _law(rng)
            tag = "fp32" if fp32 else "fp64"
            out.append((Spec(d, sig, c, lam, k, n, 90000 + 100 * seed + 10 * fp32 + j, collision=(d == 1),
                             name=f"served-{tag}[{j}] d={d} K={k} N={n}"), fp32))
    return out


def _serve(cls, mix, record_path):
    srv = cls.cls_server_create(round_histories=100_000, record_path=record_path)
    probs = [gpu_problem(s, fp32=fp32) for s, fp32 in mix]
    try:
        tickets = []
        for i, ((s, _), p) in enumerate(zip(mix, probs)):
            tickets.append(cls.cls_server_submit(srv, p, s.histories, s.seed))
            if i % 4 == 3:
                time.sleep(0.001)          # arrivals while earlier requests run
        for tk in tickets:
            assert cls.cls_server_wait(srv, tk, 120.0)
        rounds = [cls.cls_server_request_info(srv, tk)["rounds"] for tk in tickets]
        stats = cls.cls_server_get_stats(srv)
        res = [cls.cls_read_tallies(p, s.nbins) for p, (s, _) in zip(probs, mix)]
    finally:
        cls.cls_server_destroy(srv)
        for p in probs:
            cls.cls_destroy_problem(p)
    assert stats["completed"] == len(mix) and stats["failed"] == 0
    return res, rounds, stats


def test_served_requests_match_the_oracle(cls):
    mix = served_mix(1)
    cls.cls_set_launch_config(1, 1, 256, 0)       # 256 waves, chunks of <= 256 histories
    try:
        res, rounds, stats = _serve(cls, mix, record_path=0)
        res_fin, rounds_fin, _ = _serve(cls, mix, record_path=1)
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
    print("rounds", stats["rounds"], "per request", rounds, flush=True)
    # rounds were shared between requests, and each precision had rounds of
    # its own (the round of one precision is closed for the other)
    assert sum(rounds) > stats["rounds"]
    assert stats["rounds"] >= 2
    n_bins_bad = n_bins = 0
    for (s, fp32), (t, flux, fsig), (tf, fluxf, fsigf) in zip(mix, res, res_fin):
        g = tallies_dict(t)
        gf = tallies_dict(tf)
        assert g["transmitted"] + g["reflected"] + g["absorbed"] == s.histories, s.name
        # the in-kernel record equals the finalize-kernel record of the same chunks
        for k in COUNTS:
            assert g[k] == gf[k], (s.name, k)
        for k in ("T", "R", "A", "sigma_T", "sigma_R", "sigma_A"):
            assert g[k] == gf[k], (s.name, k)
        for k in ("total_flux", "sigma_total_flux"):
            assert abs(g[k] - gf[k]) <= 1e-11 * abs(gf[k]), (s.name, k)
        np.testing.assert_allclose(flux, fluxf, rtol=1e-11, atol=1e-14, err_msg=s.name)
        np.testing.assert_allclose(fsig, fsigf, rtol=1e-9, atol=1e-14, err_msg=s.name)
        if not fp32:
            o = run_oracle(s)          # same streams: the FP64 kernel follows the oracle
            for k, ok in (("transmitted", o.transmitted), ("reflected", o.reflected), ("absorbed", o.absorbed),
                          ("flights", o.flights), ("collisions", o.collisions), ("scatters", o.scatters),
                          ("interface_crossings", o.interfaces), ("lateral_reflections", o.lateral)):
                assert g[k] == ok, (s.name, k, g[k], ok)
            np.testing.assert_allclose(flux, o.flux, rtol=1e-9, atol=1e-12, err_msg=s.name)
            assert abs(g["total_flux"] - o.total_flux) <= 1e-9 * abs(o.total_flux), s.name
        else:
            o = run_oracle(s, seed=s.seed ^ 0x5DEECE66D)
            for a, sa, b, sb, name in ((g["T"], g["sigma_T"], o.T, o.sigma_T, "T"),
                                       (g["R"], g["sigma_R"], o.R, o.sigma_R, "R"),
                                       (g["A"], g["sigma_A"], o.A, o.sigma_A, "A"),
                                       (g["total_flux"], g["sigma_total_flux"], o.total_flux,
                                        o.total_flux_sigma, "flux")):
                zz = float(z(a, sa, b, sb))
                assert abs(zz) <= 4.0, (s.name, name, zz)
            n_bins_bad += int(np.sum(np.abs(z(flux, fsig, o.flux, o.flux_sigma)) > 4))
            n_bins += s.nbins
    print("FP32 served bins beyond 4 sigma", n_bins_bad, "of", n_bins, flush=True)
    assert n_bins_bad <= allowed_beyond_4(n_bins)


def test_served_finest_mesh_follows_the_oracle(cls):
    """A request at the largest mesh (CLS_MAX_BINS: its round's LDS tally buffers need
    more than 64 KB per wave) beside a small rod request, FP64 on the oracle's streams:
    counts equal and flux to 1e-9."""
    mix = [(Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), cls.CLS_MAX_BINS, 20000, 97001,
                 name="served cube at the largest mesh"), False),
           (Spec(1, (0.3, 1.2), (0.4, 0.8), (0.5, 2.0), 100, 5000, 97002, collision=True,
                 name="served rod"), False)]
    res, _, stats = _serve(cls, mix, record_path=0)
    assert stats["completed"] == 2
    for (s, _), (t, flux, _) in zip(mix, res):
        g = tallies_dict(t)
        o = run_oracle(s)
        for k, ok in (("transmitted", o.transmitted), ("reflected", o.reflected), ("absorbed", o.absorbed),
                      ("flights", o.flights), ("scatters", o.scatters), ("interface_crossings", o.interfaces),
                      ("lateral_reflections", o.lateral)):
            assert g[k] == ok, (s.name, k, g[k], ok)
        np.testing.assert_allclose(flux, o.flux, rtol=1e-9, atol=1e-12, err_msg=s.name)
