"""GPU tests of the batched, graph-captured, autotuned and served forms, the
extruded-2D and high-scattering workloads, caller-owned memory and edge cases.
All GPU calls go through the C ABI (ctypes binding)."""
from __future__ import annotations

import json
import os
import time

import numpy as np
import pytest

from helpers import (allowed_beyond_4, gpu_flags, gpu_problem, run_gpu, run_oracle, tallies_dict, z)
from paper_1708_00765_amd.inputs import Spec, workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
COUNTS = ("histories", "transmitted", "reflected", "absorbed", "flights", "collisions", "scatters",
          "interface_crossings", "lateral_reflections")


@pytest.fixture(scope="module")
def cls():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1708_00765_amd import cls as mod
    yield mod
    mod.cls_set_launch_config(0, 0, 0, 0)


def _print(*a):
    print(*a, flush=True)


def _same_results(g1, f1, g2, f2, what):
    for k in COUNTS:
        assert g1[k] == g2[k], (what, k, g1[k], g2[k])
    np.testing.assert_allclose(f1, f2, rtol=1e-11, atol=1e-13, err_msg=what)
    for k in ("T", "R", "A"):
        assert g1[k] == g2[k], (what, k)
    assert abs(g1["total_flux"] - g2["total_flux"]) <= 1e-11 * abs(g1["total_flux"]), what


# ---------------------------------------------------------------------------
# extruded 2D, 256 uneven sets in one persistent launch
# ---------------------------------------------------------------------------
def test_ext2d_batched_all_sets_vs_oracle(cls):
    specs = workload("ext2d_batched")
    cap = 40_000
    small = [Spec(s.d, s.sigma, s.c, s.lam, s.nbins, min(s.histories, cap), s.seed, name=s.name) for s in specs]
    probs = [gpu_problem(s, fp32=True) for s in small]
    try:
        cls.cls_run_batch(probs, [s.histories for s in small], [s.seed for s in small])
        res = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, small)]
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)
    n_scalar_bad = 0
    n_bins_bad = 0
    n_bins = 0
    worst = 0.0
    for s, (t, flux, fsig) in zip(small, res):
        g = tallies_dict(t)
        assert g["transmitted"] + g["reflected"] + g["absorbed"] == s.histories
        o = run_oracle(s, seed=s.seed ^ 0xABCDEF)
        for a, sa, b, sb in ((g["T"], g["sigma_T"], o.T, o.sigma_T), (g["R"], g["sigma_R"], o.R, o.sigma_R),
                             (g["total_flux"], g["sigma_total_flux"], o.total_flux, o.total_flux_sigma)):
            zz = abs(float(z(a, sa, b, sb)))
            worst = max(worst, zz)
            n_scalar_bad += zz > 4
        n_bins_bad += int(np.sum(np.abs(z(flux, fsig, o.flux, o.flux_sigma)) > 4))
        n_bins += s.nbins
    _print("ext2d: worst scalar |z|", worst, "bins beyond 4 sigma", n_bins_bad, "of", n_bins)
    assert n_scalar_bad <= allowed_beyond_4(3 * len(small))
    assert n_bins_bad <= allowed_beyond_4(n_bins)


# ---------------------------------------------------------------------------
# high-scattering 3D stress sets
# ---------------------------------------------------------------------------
def _stress_reference():
    path = os.path.join(HERE, "golden", "stress3d_oracle_1e6.json")
    if not os.path.exists(path):
        pytest.skip("stress3d oracle reference not generated")
    return json.load(open(path))["sets"]


@pytest.mark.parametrize("fp32", [True, False])
def test_stress3d_vs_oracle_reference(cls, fp32):
    ref = _stress_reference()
    specs = workload("stress3d", histories=4_000_000)
    probs = [gpu_problem(s, fp32=fp32) for s in specs]
    try:
        cls.cls_run_batch(probs, [s.histories for s in specs], [s.seed for s in specs])
        res = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)
    bad = 0
    nb_bad = 0
    nb = 0
    worst = 0.0
    for s, r, (t, flux, fsig) in zip(specs, ref, res):
        assert r["name"] == s.name and tuple(r["sigma"]) == tuple(s.sigma)
        g = tallies_dict(t)
        assert g["capped"] == 0
        for k, sk in (("T", "sigma_T"), ("R", "sigma_R"), ("total_flux", "sigma_total_flux")):
            zz = abs(float(z(g[k], g[sk], r[k], r[sk])))
            worst = max(worst, zz)
            bad += zz > 4
        if "flux" in r:
            nb_bad += int(np.sum(np.abs(z(flux, fsig, np.array(r["flux"]), np.array(r["flux_sigma"]))) > 4))
            nb += len(r["flux"])
    _print("stress3d", "fp32" if fp32 else "fp64", "worst |z|", worst, "bins beyond 4 sigma", nb_bad, "of", nb)
    assert bad <= allowed_beyond_4(3 * len(specs))
    assert nb > 0 and nb_bad <= allowed_beyond_4(nb)


def test_stress3d_fp32_deviation_from_fp64(cls):
    """Common random numbers: FP32 tracking vs FP64 tracking on the same streams."""
    specs = workload("stress3d", histories=2_000_000)
    out = {}
    for fp32 in (False, True):
        probs = [gpu_problem(s, fp32=fp32) for s in specs]
        try:
            cls.cls_run_batch(probs, [s.histories for s in specs], [s.seed for s in specs])
            out[fp32] = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
        finally:
            for p in probs:
                cls.cls_destroy_problem(p)
    worst_rel = 0.0
    worst_sig = 0.0
    for (t64, f64, s64), (t32, f32, _) in zip(out[False], out[True]):
        for k, sk in (("T", "sigma_T"), ("R", "sigma_R"), ("total_flux", "sigma_total_flux")):
            a, b, sg = getattr(t64, k), getattr(t32, k), getattr(t64, sk)
            worst_rel = max(worst_rel, abs(a - b) / max(abs(a), 1e-300))
            worst_sig = max(worst_sig, abs(a - b) / max(sg, 1e-300))
    _print("stress3d fp32 vs fp64: worst relative deviation", worst_rel, "worst in sigma", worst_sig)
    assert worst_sig < 1.0


# ---------------------------------------------------------------------------
# graphs, autotuning, caller memory
# ---------------------------------------------------------------------------
def test_graph_replays_match_eager_runs(cls):
    specs = workload("cube3d_track", histories=500_000)
    eager = [gpu_problem(s, fp32=True) for s in specs]
    graph = [gpu_problem(s, fp32=True) for s in specs]
    b = cls.cls_batch_create(graph)
    try:
        for k in range(4):
            seeds = [s.seed + 1000 * k for s in specs]
            hist = [s.histories - 977 * k for s in specs]
            cls.cls_batch_run(b, hist, seeds)
            # the program's own eager work between replays
            cls.cls_run_batch(eager, hist, seeds)
            for s, pe, pg in zip(specs, eager, graph):
                te, fe, _ = cls.cls_read_tallies(pe, s.nbins)
                tg, fg, _ = cls.cls_read_tallies(pg, s.nbins)
                _same_results(tallies_dict(te), fe, tallies_dict(tg), fg, f"replay {k} {s.name}")
        assert cls.cls_batch_last_ms(b) > 0
    finally:
        cls.cls_batch_destroy(b)
        for p in eager + graph:
            cls.cls_destroy_problem(p)


def test_ext2d_full_size_launch_shape_follows_the_oracle_fp64(cls):
    """The twelve finest extruded meshes (up to 998 bins) with the full-size batch's
    launch configuration (one LDS tally buffer per wave, the autotuner's 65536-history
    chunk cap; the chunks themselves follow these smaller history counts), FP64 on the
    oracle's streams at history counts the oracle finishes in seconds: counts equal and
    flux to 1e-9 for every set."""
    specs = workload("ext2d_batched")
    sub = [Spec(s.d, s.sigma, s.c, s.lam, s.nbins, min(s.histories, 20_000), s.seed, name=s.name)
           for s in sorted(specs, key=lambda s: -s.nbins)[:12]]
    probs = [gpu_problem(s, fp32=False) for s in sub]
    cls.cls_set_launch_config(max_chunk=65536, slots=1)
    try:
        cls.cls_run_batch(probs, [s.histories for s in sub], [s.seed for s in sub])
        res = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, sub)]
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
        for p in probs:
            cls.cls_destroy_problem(p)
    for s, (t, flux, _) in zip(sub, res):
        g = tallies_dict(t)
        o = run_oracle(s)
        for key, ok in (("transmitted", o.transmitted), ("reflected", o.reflected), ("absorbed", o.absorbed),
                        ("flights", o.flights), ("scatters", o.scatters), ("interface_crossings", o.interfaces),
                        ("lateral_reflections", o.lateral)):
            assert g[key] == ok, (s.name, key, g[key], ok)
        np.testing.assert_allclose(flux, o.flux, rtol=1e-9, atol=1e-12, err_msg=s.name)


def test_graph_replays_follow_the_oracle_fp64(cls):
    """FP64 graph replays on the oracle's streams (Algorithm A, Section 4): every replay,
    with new history counts and seeds, gives the oracle's counts exactly and its flux
    to 1e-9."""
    specs = workload("cube3d_track", histories=20_000)[:3]
    graph = [gpu_problem(s, fp32=False) for s in specs]
    b = cls.cls_batch_create(graph)
    try:
        for k in range(2):
            seeds = [s.seed + 7919 * (k + 1) for s in specs]
            hist = [s.histories - 331 * k for s in specs]
            cls.cls_batch_run(b, hist, seeds)
            for s, p, n, sd in zip(specs, graph, hist, seeds):
                t, flux, _ = cls.cls_read_tallies(p, s.nbins)
                g = tallies_dict(t)
                o = run_oracle(s, histories=n, seed=sd)
                for key, ok in (("transmitted", o.transmitted), ("reflected", o.reflected),
                                ("absorbed", o.absorbed), ("flights", o.flights), ("scatters", o.scatters),
                                ("interface_crossings", o.interfaces), ("lateral_reflections", o.lateral)):
                    assert g[key] == ok, (k, s.name, key, g[key], ok)
                np.testing.assert_allclose(flux, o.flux, rtol=1e-9, atol=1e-12, err_msg=f"replay {k} {s.name}")
    finally:
        cls.cls_batch_destroy(b)
        for p in graph:
            cls.cls_destroy_problem(p)


@pytest.mark.parametrize("fp32", [True, False])
def test_results_do_not_depend_on_launch_shape_and_autotune(cls, fp32):
    """Counts exactly, score and flux sums to FP64 summation order, for launch
    shapes from one-wave workgroups with 64-history chunks refilled lane by
    lane (a lane changes chunk slot after almost every history) to 65536-history
    chunks, with one or two LDS tally buffers per wave forced; then the
    autotuner's choice (FP32)."""
    specs = workload("cube3d_track", histories=300_000)[:4]
    probs = [gpu_problem(s, fp32=fp32) for s in specs]
    hist = [s.histories for s in specs]
    seeds = [s.seed for s in specs]
    try:
        cls.cls_run_batch(probs, hist, seeds)
        base = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
        for cfg in ((1, 1, 64, 1, 0), (8, 0, 1024, 16, 0), (2, 3, 65536, 4, 0), (0, 0, 4096, 4, 1),
                    (0, 0, 4096, 4, 2)):
            cls.cls_set_launch_config(*cfg)
            cls.cls_run_batch(probs, hist, seeds)
            for s, p, (t0, f0, _) in zip(specs, probs, base):
                t1, f1, _ = cls.cls_read_tallies(p, s.nbins)
                # counts are exact; the flux sums only change by atomic ordering
                for k in COUNTS:
                    assert getattr(t0, k) == getattr(t1, k), (cfg, k)
                for k in ("total_flux", "sigma_total_flux"):
                    assert abs(getattr(t0, k) - getattr(t1, k)) <= 1e-11 * abs(getattr(t0, k)), (cfg, k)
                np.testing.assert_allclose(f0, f1, rtol=1e-11, atol=1e-13)
        cls.cls_set_launch_config(0, 0, 0, 0)
        if not fp32:
            return
        cfg, rate = cls.cls_autotune(probs, hist, sample_histories=2_000_000)
        _print("autotuned", cfg, rate)
        assert cfg["waves_per_block"] in (0, 1, 2, 4, 8) and rate > 0
        cls.cls_run_batch(probs, hist, seeds)
        for s, p, (t0, _, _) in zip(specs, probs, base):
            t1, _, _ = cls.cls_read_tallies(p, s.nbins)
            assert t0.transmitted == t1.transmitted and t0.flights == t1.flights
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
        for p in probs:
            cls.cls_destroy_problem(p)


def test_batch_chunks_keep_error_batches(cls):
    """A problem keeps at least min(256, n / 64) batches of its per-bin flux
    error, in a batch of problems as alone; counts stay those of the lone run."""
    specs = workload("ext2d_batched", histories=None)[:24]
    alone = [run_gpu(s, fp32=True)[0] for s in specs]
    probs = [gpu_problem(s, fp32=True) for s in specs]
    try:
        cls.cls_run_batch(probs, [s.histories for s in specs], [s.seed for s in specs])
        for s, p, g1 in zip(specs, probs, alone):
            t, _, fsig = cls.cls_read_tallies(p, s.nbins)
            g2 = tallies_dict(t)
            _print(s.name, "histories", s.histories, "chunks alone", g1["batches"], "in the batch", g2["batches"])
            assert min(g1["batches"], g2["batches"]) >= min(256, s.histories // 64), s.name
            for k in COUNTS:
                assert g1[k] == g2[k], (s.name, k)
            assert np.all(np.isfinite(fsig))
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)


def _fine_mesh_mix(big_histories, n_big, n_small, seed):
    """n_big cube3d problems with 700-1000 bins and big_histories each, plus
    n_small problems of 1e3 to 1e5 histories and 10 to 1000 bins (FP32)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_big + n_small):
        sig = tuple(float(v) for v in rng.uniform(0.2, 2.0, 2))
        c = tuple(float(v) for v in rng.uniform(0.0, 0.95, 2))
        lam = tuple(float(v) for v in rng.uniform(0.2, 5.0, 2))
        if i < n_big:
            k, n = int(rng.integers(700, 1001)), big_histories
        else:
            k, n = int(rng.integers(10, 1001)), int(10 ** rng.uniform(3, 5))
        specs.append(Spec(3, sig, c, lam, k, n, 7000 + seed * 100 + i, name=f"mix{seed}[{i}]"))
    return specs


def test_fine_mesh_batch_with_tiny_problems_equals_single_runs(cls):
    """Fine meshes in a batch whose histories sit almost all in chunks of
    thousands of histories: the launch keeps one LDS tally buffer per wave even
    though a few problems are tiny (their chunks hold tens of histories). Every
    problem gets the tallies of its lone run: counts exactly, flux to FP64
    summation order."""
    specs = _fine_mesh_mix(160_000_000, 2, 8, seed=1)
    _print("fine-mesh batch:", [(s.histories, s.nbins) for s in specs])
    probs = [gpu_problem(s, fp32=True) for s in specs]
    try:
        cls.cls_run_batch(probs, [s.histories for s in specs], [s.seed for s in specs])
        batched = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
        for s, p, (tb, fb, sb) in zip(specs, probs, batched):
            cls.cls_run(p, s.histories, s.seed)
            ta, fa, _ = cls.cls_read_tallies(p, s.nbins)
            _same_results(tallies_dict(ta), fa, tallies_dict(tb), fb, s.name)
            assert np.all(np.isfinite(sb)), s.name
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)


def test_served_small_requests_overtake_big_ones_and_keep_results(cls):
    """Two big fine-mesh requests (1.2e9 histories each) submitted first, then a few
    tiny ones: the tiny requests go to the priority queue of the round already on
    the GPU and complete long before the big ones; each result equals its lone run
    (counts exactly, flux to summation order)."""
    specs = _fine_mesh_mix(1_200_000_000, 2, 6, seed=2)
    _print("served mix:", [(s.histories, s.nbins) for s in specs])
    probs = [gpu_problem(s, fp32=True) for s in specs]
    srv = cls.cls_server_create()
    try:
        tickets = [cls.cls_server_submit(srv, p, s.histories, s.seed) for s, p in zip(specs, probs)]
        for tk in tickets:
            assert cls.cls_server_wait(srv, tk, 120.0)
        infos = [cls.cls_server_request_info(srv, tk) for tk in tickets]
        stats = cls.cls_server_get_stats(srv)
        _print("server stats", stats, "latency ms", [round(1e3 * (i["done_s"] - i["submit_s"]), 2) for i in infos])
        assert stats["completed"] == len(specs) and stats["failed"] == 0
        big_done = min(i["done_s"] for i in infos[:2])
        assert all(i["done_s"] < big_done for i in infos[2:])      # tiny requests overtake
        served = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
    finally:
        cls.cls_server_destroy(srv)
    try:
        for s, p, (tm, fm, _) in zip(specs, probs, served):
            cls.cls_run(p, s.histories, s.seed)
            ta, fa, _ = cls.cls_read_tallies(p, s.nbins)
            _same_results(tallies_dict(ta), fa, tallies_dict(tm), fm, s.name)
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)


def test_gathered_error_batches(cls):
    """A wave gathers the chunks it takes of one problem into one error batch
    (default) instead of flushing every chunk (chunk_batches = 1): on the cube
    workload (8 sets, 2e6 histories each) the counts are equal, the flux agrees
    to summation order, every set keeps at least 256 batches and no more than
    chunks, the sets together have at most half as many batches as chunks, and
    the per-bin batch-means errors of the two batchings agree within their
    statistical spread."""
    specs = workload("cube3d_track", histories=2_000_000)
    probs = [gpu_problem(s, fp32=True) for s in specs]
    out = {}
    try:
        for cb in (1, 0):
            cls.cls_set_launch_config(chunk_batches=cb)
            cls.cls_run_batch(probs, [s.histories for s in specs], [s.seed for s in specs])
            out[cb] = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
        for p in probs:
            cls.cls_destroy_problem(p)
    for s, (t1, f1, e1), (t0, f0, e0) in zip(specs, out[1], out[0]):
        g1, g0 = tallies_dict(t1), tallies_dict(t0)
        for k in COUNTS:
            assert g1[k] == g0[k], (s.name, k)
        np.testing.assert_allclose(f0, f1, rtol=1e-11, atol=1e-13, err_msg=s.name)
        assert g0["total_flux"] == pytest.approx(g1["total_flux"], rel=1e-11)
        assert g0["sigma_total_flux"] == pytest.approx(g1["sigma_total_flux"], rel=1e-11)
        _print(s.name, "chunks", g1["batches"], "gathered batches", g0["batches"])
        assert 256 <= g0["batches"] <= g1["batches"], s.name
        assert np.array_equal(e1 > 0, e0 > 0), s.name
        ratio = e0[e1 > 0] / e1[e1 > 0]
        # the spread of a batch-means error is about 1 / sqrt(2 (B - 1)) where
        # many histories reach the bin (relative error below 1%); in sparsely
        # reached bins it is set by the few histories that score there
        dense = (e1 > 0) & (e1 < 0.01 * np.abs(f1))
        rd = e0[dense] / e1[dense]
        tol = 8.0 / np.sqrt(2.0 * (g0["batches"] - 1))
        _print(s.name, "flux sigma ratio: all bins", ratio.min(), np.median(ratio), ratio.max(), "dense bins",
               int(dense.sum()), rd.min(), rd.max(), "tolerance", tol)
        assert dense.sum() >= 10, s.name
        assert np.all(np.abs(rd - 1.0) <= tol), s.name
        assert abs(np.median(ratio) - 1.0) <= 0.05, s.name
    n_chunks = sum(t.batches for t, _, _ in out[1])
    n_gathered = sum(t.batches for t, _, _ in out[0])
    _print("chunks", n_chunks, "gathered batches", n_gathered)
    assert n_gathered <= n_chunks // 2


def test_single_tally_buffer_mode_matches_oracle(cls):
    """A 1000-bin mesh with chunks of at least 2048 histories runs with one LDS
    tally buffer per wave (more waves resident than with two); with chunks of
    at most 1024 histories the same problem runs with two buffers. Both give
    the oracle's counts exactly (FP64 on the same streams) and its flux to
    rounding (the chunking changes the order of the sums). Every chunk is its
    own error batch here, so that the batch count shows the chunk size."""
    s = Spec(1, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 1000, 48_000_000, 31)
    _print("single-buffer case: rod, 1000 bins, 4.8e7 histories")
    o = run_oracle(s)
    results = []
    try:
        for max_chunk in (0, 1024):
            cls.cls_set_launch_config(0, 0, max_chunk, 0, chunk_batches=1)
            g, flux, _, _ = run_gpu(s)
            _print("max_chunk", max_chunk, "histories per chunk", g["histories"] / g["batches"])
            results.append((g, flux))
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
    (g1, f1), (g2, f2) = results
    assert g1["histories"] / g1["batches"] >= 2048 and g2["histories"] / g2["batches"] <= 1024
    for g, f in results:
        for k, ok in (("transmitted", o.transmitted), ("reflected", o.reflected), ("absorbed", o.absorbed),
                      ("flights", o.flights), ("collisions", o.collisions), ("scatters", o.scatters),
                      ("interface_crossings", o.interfaces)):
            assert g[k] == ok, k
        np.testing.assert_allclose(f, o.flux, rtol=1e-9, atol=1e-12)


def test_caller_owned_memory_and_stream(cls):
    import torch
    s = workload("cube3d_track", histories=200_000)[2]
    g_ref, f_ref, _, _ = run_gpu(s, fp32=True)
    p = gpu_problem(s, fp32=True)
    try:
        nbytes = cls.cls_footprint(p, s.histories)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = (buf.data_ptr() + 255) // 256 * 256
        cls.cls_bind_device_memory(p, ptr, nbytes)
        stream = torch.cuda.Stream()
        cls.cls_set_stream(p, stream.cuda_stream)
        cls.cls_run_async(p, s.histories, s.seed)
        cls.cls_synchronize(p)
        t, f, _ = cls.cls_read_tallies(p, s.nbins)
        _same_results(g_ref, f_ref, tallies_dict(t), f, "bound memory")
        with pytest.raises(cls.ClsError):
            cls.cls_bind_device_memory(p, ptr + 8, nbytes)     # misaligned
    finally:
        cls.cls_destroy_problem(p)


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
def _served_specs(n, seed=5):
    from paper_1708_00765_amd.inputs import served_requests
    reqs = served_requests(rate_hz=1000.0, duration_s=1.0, salt=seed, max_histories=3e6)
    return [s for _, s in reqs[:n]]


def test_served_results_equal_alone_and_in_the_mix(cls):
    """A big request keeps the GPU busy while 40 mixed requests arrive: they
    share rounds (more request-rounds than rounds), and every result equals
    the same request run alone (counts exactly, FP64 sums to 1e-11)."""
    big = Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 200, 300_000_000, 4242, name="served-big")
    specs = [big] + _served_specs(40)
    srv = cls.cls_server_create(round_histories=2_000_000)
    probs = [gpu_problem(s, fp32=True) for s in specs]
    try:
        tickets = []
        for i, (s, p) in enumerate(zip(specs, probs)):
            tickets.append(cls.cls_server_submit(srv, p, s.histories, s.seed))
            if i % 7 == 0:
                time.sleep(0.002)          # arrivals while earlier requests run
        for tk in tickets:
            assert cls.cls_server_wait(srv, tk, 120.0)
        mixed = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
        stats = cls.cls_server_get_stats(srv)
        per_request = [cls.cls_server_request_info(srv, tk)["rounds"] for tk in tickets]
        _print("server stats", stats, "request-rounds", sum(per_request))
        assert stats["completed"] == len(specs) and stats["failed"] == 0
        assert sum(per_request) > stats["rounds"]   # some rounds carried several requests
        _print("requests spread over several rounds:", sum(r > 1 for r in per_request))
    finally:
        cls.cls_server_destroy(srv)
    for s, p, (tm, fm, _) in zip(specs, probs, mixed):
        cls.cls_run(p, s.histories, s.seed)
        ta, fa, _ = cls.cls_read_tallies(p, s.nbins)
        _same_results(tallies_dict(ta), fa, tallies_dict(tm), fm, s.name)
        cls.cls_destroy_problem(p)


def test_server_admission_respects_the_budget(cls):
    specs = _served_specs(12, seed=9)
    probs = [gpu_problem(s, fp32=True) for s in specs]
    fp = max(cls.cls_footprint(p, s.histories) for p, s in zip(probs, specs))
    srv = cls.cls_server_create(hbm_budget_bytes=2 * fp, round_histories=500_000)
    try:
        tickets = [cls.cls_server_submit(srv, p, s.histories, s.seed) for s, p in zip(specs, probs)]
        with pytest.raises(cls.ClsError):         # one request per problem at a time
            cls.cls_server_submit(srv, probs[-1], 100, 1)
        for tk in tickets:
            assert cls.cls_server_wait(srv, tk, 120.0)
        st = cls.cls_server_get_stats(srv)
        assert st["hbm_peak"] <= 2 * fp and st["completed"] == len(specs)
        for tk in tickets:
            info = cls.cls_server_request_info(srv, tk)
            assert info["submit_s"] <= info["admit_s"] <= info["done_s"]
            cls.cls_server_release(srv, tk)
        with pytest.raises(cls.ClsError):
            cls.cls_server_poll(srv, tickets[0])   # released
    finally:
        cls.cls_server_destroy(srv)
        for p in probs:
            cls.cls_destroy_problem(p)


def test_server_budget_bounds_device_memory(cls):
    """600 pending requests with 2000-bin meshes (~36 KB of tallies each, ~21 MB in
    all) behind a big one, under a 4 MB budget: the device memory the server holds
    (hipMemGetInfo, while they wait) stays within the budget plus its fixed round
    buffers and the allocator's rounding (8 MB, against ~21 MB for all of them),
    and every request completes."""
    import torch
    torch.cuda.synchronize()
    big = Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 2000, 200_000_000, 4343, name="budget-big")
    smalls = [Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 2000, 2000, 5000 + i, name=f"budget[{i}]")
              for i in range(600)]
    specs = [big] + smalls
    probs = [gpu_problem(s, fp32=True) for s in specs]
    budget = 4 << 20
    free0, _ = torch.cuda.mem_get_info()
    srv = cls.cls_server_create(hbm_budget_bytes=budget)
    try:
        tickets = [cls.cls_server_submit(srv, p, s.histories, s.seed) for s, p in zip(specs, probs)]
        time.sleep(0.05)
        free1, _ = torch.cuda.mem_get_info()
        st = cls.cls_server_get_stats(srv)
        _print("device memory held by the server", free0 - free1, "budget", budget, "pending", st["pending"])
        assert free0 - free1 <= budget + (8 << 20)
        for tk in tickets:
            assert cls.cls_server_wait(srv, tk, 120.0)
        st = cls.cls_server_get_stats(srv)
        assert st["completed"] == len(specs) and st["failed"] == 0 and st["hbm_peak"] <= budget
    finally:
        cls.cls_server_destroy(srv)
        for p in probs:
            cls.cls_destroy_problem(p)


# ---------------------------------------------------------------------------
# edge cases (FP64 on the oracle's streams: identical counts)
# ---------------------------------------------------------------------------
EDGE = [
    ("one history", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 50, 1, 11)),
    ("ragged tail 63", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 50, 63, 12)),
    ("ragged tail 65", Spec(2, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 50, 65, 13)),
    ("ragged 4099", Spec(1, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 37, 4099, 14, collision=True)),
    ("one bin", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 1, 5000, 15)),
    ("max bins", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 8192, 5000, 16)),
    ("max bins in 64 KB", Spec(2, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 8100, 3000, 26)),
    ("pure absorber", Spec(3, (0.5, 1.5), (0.0, 0.0), (1.0, 0.3), 100, 5000, 17)),
    ("pure scatterer", Spec(2, (0.5, 1.5), (1.0, 1.0), (1.0, 0.3), 100, 5000, 18)),
    ("optically thin", Spec(3, (1e-4, 1e-4), (0.5, 0.5), (1e6, 1e6), 100, 5000, 19)),
    ("tiny chords", Spec(1, (0.5, 1.5), (0.5, 0.9), (1e-3, 2e-3), 100, 2000, 20, collision=True)),
    ("slab volume source", Spec(1, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 100, 5000, 21, slab=True, source=1)),
    ("cube volume source", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 100, 5000, 22, source=1)),
    ("2D volume source", Spec(2, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 100, 5000, 23, source=1)),
    ("rod volume source", Spec(1, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 100, 5000, 24, source=1, collision=True)),
    ("short box", Spec(3, (0.5, 1.5), (0.5, 0.9), (1.0, 0.3), 10, 5000, 25, L=0.1)),
]


@pytest.mark.parametrize("name,s", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases_follow_the_oracle(cls, name, s):
    _print("case", name)
    g, flux, _, (hsh, fl) = run_gpu(s, trace_n=s.histories)
    o = run_oracle(s, trace=True)
    assert g["transmitted"] + g["reflected"] + g["absorbed"] + g["capped"] == s.histories
    same = float(np.mean(hsh == o.trace_hash))
    assert same >= 0.999, same
    if same == 1.0:
        for k, ok in (("transmitted", o.transmitted), ("reflected", o.reflected), ("absorbed", o.absorbed),
                      ("flights", o.flights), ("collisions", o.collisions), ("scatters", o.scatters),
                      ("interface_crossings", o.interfaces), ("lateral_reflections", o.lateral)):
            assert g[k] == ok, (name, k)
        np.testing.assert_allclose(flux, o.flux, rtol=1e-9, atol=1e-12)
