#!/usr/bin/env python3
"""Throughput of Chord Length Sampling (Algorithm A, arXiv 1708.00765 Section 4)
on one MI355X.

Default workload (stress3d, the divergence-stress configuration): d=3 cube of side
10, vacuum x-faces, mirroring lateral faces, cosine-weighted incidence on x=0; 32
seeded parameter sets in the high-scattering, optically thick regime (c_i uniform in
[0.99, 0.999], Sigma_i log-uniform in [0.5, 5], Lambda_i log-uniform in [0.05, 1]);
1e8 histories per set; 1000 x-bins with the track-length estimator. A step runs all
32 sets in one batched persistent launch with FP32 flight arithmetic, FP64 positions
and FP64 tallies, then finalizes and copies the results back.

Also reported: the plain FP64 one-problem-per-launch rate on the same sets and the
FP32 form's deviation from it on the same random streams (the acceptance rule of the
FP32 form), the roofline of the tracking kernel (VALU issue slots, see perf_model.py),
the FP64 CPU oracle on a bounded sample of the same sets (and each set's FP32 result
against that oracle sample in combined standard deviations), the cube3d and extruded
2D workloads, the quenched d = 1 kernel and the served Poisson request stream.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(cls, s, fp32):
    flags = (cls.CLS_F_FP32 if fp32 else 0) | (cls.CLS_F_COLLISION_FLUX if s.collision else 0) | \
            (cls.CLS_F_D1_SLAB if s.slab else 0)
    return cls.cls_create_problem(s.d, s.L, s.sigma, s.c, s.lam, source=s.source, nbins=s.nbins, flags=flags)


def run_batch_steps(cls, torch, probs, specs, steps, warmup, seed_salt):
    hist = [s.histories for s in specs]

    def seeds(k):
        return [(s.seed + 0x9E3779B97F4A7C15 * (k + seed_salt)) & (2**64 - 1) for s in specs]

    for k in range(warmup):
        cls.cls_run_batch(probs, hist, seeds(k))
    torch.cuda.synchronize()
    track_ms = 0.0
    t0 = time.perf_counter()
    for k in range(steps):
        cls.cls_run_batch(probs, hist, seeds(warmup + k))
        t, _, _ = cls.cls_read_tallies(probs[0], specs[0].nbins)
        track_ms += t.track_ms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    full = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs, specs)]
    return wall, track_ms, full


def kernel_source_sha256():
    """Hash of the tracking kernel's sources (the kernel and the headers it includes)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("cls_track.hip", "cls_internal.hpp", "philox.hpp"):
        with open(os.path.join(ROOT, "paper_1708_00765_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name):
    """HBM bytes per tracking launch of a workload from its committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"track_kernel_{workload_name}_traffic.md")
    if not os.path.exists(path):
        return None
    keys = {}
    for line in open(path):
        parts = line.strip().split(":", 1)
        if len(parts) == 2 and parts[0] in ("kernel_source_sha256", "traffic_bytes_per_launch"):
            keys[parts[0]] = parts[1].strip()
    if keys.get("kernel_source_sha256") != kernel_source_sha256() or "traffic_bytes_per_launch" not in keys:
        return None
    return float(keys["traffic_bytes_per_launch"])


# Acceptance rule of the FP32 form (fixed before it was measured), per parameter set,
# with x32 / x64 the FP32 / FP64 results on the same random streams and sigma64 the
# FP64 one-sigma error: (1) T, R, A and the total flux within 1e-4 relative; (2) the
# flux profile within 1e-4 in L2 norm; (3) every bin within 1e-4 relative plus a tenth
# of the bin's FP64 sigma. No set and no bin is left out.
RULE_REL = 1e-4
RULE_SIGMA_SHARE = 0.1


def fp32_acceptance(full32, full64):
    """Evaluate the acceptance rule over all sets: worst values and violation counts."""
    import numpy as np
    worst_s = worst_p = worst_b = worst_sig = 0.0
    v_s = v_p = v_b = 0
    for (t32, f32, _), (t64, f64, s64) in zip(full32, full64):
        for k, sk in (("T", "sigma_T"), ("R", "sigma_R"), ("A", "sigma_A"), ("total_flux", "sigma_total_flux")):
            a, b, sg = getattr(t64, k), getattr(t32, k), getattr(t64, sk)
            r = abs(b - a) / abs(a) if a != 0.0 else (0.0 if b == a else float("inf"))
            worst_s = max(worst_s, r)
            v_s += r > RULE_REL
            if sg > 0.0:
                worst_sig = max(worst_sig, abs(b - a) / sg)
        n64 = float(np.linalg.norm(f64))
        if n64 > 0.0:
            r = float(np.linalg.norm(f32 - f64)) / n64
            worst_p = max(worst_p, r)
            v_p += r > RULE_REL
        bound = RULE_REL * np.abs(f64) + RULE_SIGMA_SHARE * s64
        diff = np.abs(f32 - f64)
        v_b += int(np.sum(diff > bound))
        ok = bound > 0
        if ok.any():
            worst_b = max(worst_b, float(np.max(diff[ok] / bound[ok])))
    return {"max_rel_scalar": worst_s, "max_rel_profile_l2": worst_p, "max_bin_deviation_over_allowance": worst_b,
            "max_scalar_deviation_in_fp64_sigma": worst_sig,
            "violations": {"scalars": v_s, "profiles": v_p, "bins": v_b},
            "bins_compared": int(sum(len(f[1]) for f in full64)),
            "passes": v_s == 0 and v_p == 0 and v_b == 0,
            "rule": "per set: T, R, A, total flux within 1e-4 relative; flux profile within 1e-4 (L2); "
                    "every bin within 1e-4 relative + 0.1 FP64 sigma; FP32 vs FP64 on the same streams"}


def oracle_agreement(full32, oracle_results):
    """Each set's FP32 GPU result against the FP64 oracle on independent streams, in
    combined standard deviations: the worst |z| of T, R, A and the total flux, and the
    flux bins beyond 4 sigma against the 0.999 quantile of Binomial(bins, 6.3e-5)."""
    import numpy as np
    from scipy.stats import binom
    zmax = 0.0
    beyond = bins = 0
    for (t, f, fs), o in zip(full32, oracle_results):
        for a, sa, b, sb in ((t.T, t.sigma_T, o.T, o.sigma_T), (t.R, t.sigma_R, o.R, o.sigma_R),
                             (t.A, t.sigma_A, o.A, o.sigma_A),
                             (t.total_flux, t.sigma_total_flux, o.total_flux, o.total_flux_sigma)):
            sc = (sa * sa + sb * sb) ** 0.5
            if sc > 0:
                zmax = max(zmax, abs(a - b) / sc)
        sc = np.hypot(fs, o.flux_sigma)
        ok = sc > 0
        beyond += int(np.sum(np.abs(f[ok] - o.flux[ok]) / sc[ok] > 4.0))
        bins += int(ok.sum())
    return {"max_abs_z_scalars": zmax, "bins_beyond_4_sigma": beyond, "bins": bins,
            "bins_beyond_4_sigma_allowed": int(binom.ppf(0.999, max(bins, 1), 6.334e-5)),
            "oracle_histories_per_set": int(oracle_results[0].histories) if oracle_results else 0}


def load_paper_rows():
    """The CLS rows of Tables 3-8 (printed values, one-sigma errors and t_tot)."""
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_cls_rows.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "I":
            vals = {"R": (float(f[3]), float(f[4])), "T": (float(f[5]), float(f[6])),
                    "flux": (float(f[7]), float(f[8]))}
            t_tot = float(f[9])
        else:
            vals = {"Lk": (float(f[3]), float(f[4])), "flux": (float(f[5]), float(f[6]))}
            t_tot = float(f[7])
        rows.append((f[0], f[1], int(f[2]), vals, t_tot, f[-1]))
    return rows


def run_paper_rows(cls, torch, stream, histories, fp32):
    """Every CLS row of Tables 3-8 as one plain run of `histories` histories:
    the paper's observables (suite I: R, T, <phi>; suite II: the leakage
    <(T+R)/2> and <phi>) against the printed values, in combined standard
    deviations, and the GPU time of the run against the printed t_tot."""
    import math
    from paper_1708_00765_amd.inputs import paper_case
    out = []
    for i, (suite, case, d, vals, t_tot, table) in enumerate(load_paper_rows()):
        s = paper_case(case, d, suite, histories=histories, seed=770000 + i)
        p = make_problem(cls, s, fp32)
        cls.cls_set_stream(p, stream)
        cls.cls_run(p, min(histories, 100_000), s.seed + 1)      # warm the code object
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cls.cls_run(p, histories, s.seed)
        t, _, _ = cls.cls_read_tallies(p, s.nbins)
        wall = time.perf_counter() - t0
        cls.cls_destroy_problem(p)
        n = t.histories
        if suite == "I":
            obs = {"R": (t.R, t.sigma_R), "T": (t.T, t.sigma_T), "flux": (t.total_flux, t.sigma_total_flux)}
        else:
            leaked = t.transmitted + t.reflected
            mean = 0.5 * leaked / n
            var = (0.25 * leaked / n - mean * mean) * n / (n - 1)
            obs = {"Lk": (mean, math.sqrt(max(var, 0.0) / n)), "flux": (t.total_flux, t.sigma_total_flux)}
        zs = {}
        for k, (v, sv) in vals.items():
            m, sm = obs[k]
            zs[k] = (m - v) / math.sqrt(sm * sm + sv * sv)
        out.append({"table": table, "suite": suite, "case": case, "d": d, "histories": n,
                    "ours": {k: obs[k][0] for k in vals}, "ours_sigma": {k: obs[k][1] for k in vals},
                    "paper": {k: vals[k][0] for k in vals}, "z": zs,
                    "gpu_s": wall, "kernel_s": t.track_ms * 1e-3, "paper_t_tot_s": t_tot})
        log(f"  {table} {suite:2s} {case} d={d}: " + ", ".join(f"{k} z={zs[k]:+.2f}" for k in zs)
            + f"; {wall:.2f} s (paper t_tot {t_tot:.3g} s)")
    return out


def paper_realizations(suite, case):
    """Realizations per d = 1 reference row (Sec. 3.3): 4e4 for sub-cases 1b,
    5e4 for 2b, 1e5 for 3b, 5e4 for suite II 2a, 1e4 otherwise."""
    if case == "1b":
        return 40_000
    if case == "2b" or (suite == "II" and case == "2a"):
        return 50_000
    if case == "3b":
        return 100_000
    return 10_000


def load_paper_ref_rows():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_ref_rows.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "I":
            vals = {"R": (float(f[3]), float(f[4])), "T": (float(f[5]), float(f[6])),
                    "flux": (float(f[7]), float(f[8]))}
            t_tot = float(f[9])
        else:
            vals = {"Lk": (float(f[3]), float(f[4])), "flux": (float(f[5]), float(f[6]))}
            t_tot = float(f[7])
        rows.append((f[0], f[1], int(f[2]), vals, t_tot, f[-1]))
    return rows


def run_paper_ref_rows(cls, torch, stream, histories, cls_histories):
    """The d = 1 quenched reference rows of Tables 3-8 on the GPU: the paper's
    ensemble size per row (Sec. 3.3) with `histories` histories per
    realization, against the printed Ref values; and, with cls_histories > 0,
    the CLS error (CLS - Ref) / Ref of this GPU's own CLS and reference runs
    against the paper's CLS and Ref rows."""
    import math
    from paper_1708_00765_amd.inputs import paper_case
    cls_rows = {(r[0], r[1], r[2]): r[3] for r in load_paper_rows()}
    out = []
    for i, (suite, case, d, vals, t_tot, table) in enumerate(load_paper_ref_rows()):
        if d != 1:
            continue
        s = paper_case(case, 1, suite, histories=1, seed=990000 + i)
        p = make_problem(cls, s, False)
        cls.cls_set_stream(p, stream)
        M = paper_realizations(suite, case)
        cls.cls_run_quenched(p, 10, 10, s.seed + 1)                # warm the code object
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cls.cls_run_quenched(p, M, histories, s.seed)
        g, _, _ = cls.cls_read_quenched(p, s.nbins)
        wall = time.perf_counter() - t0
        cls.cls_destroy_problem(p)
        obs = {"R": (g.R, g.sigma_R), "T": (g.T, g.sigma_T), "flux": (g.total_flux, g.sigma_total_flux),
               "Lk": (g.Lk, g.sigma_Lk)}
        zs = {k: (obs[k][0] - v) / math.hypot(obs[k][1], sv) for k, (v, sv) in vals.items()}
        row = {"table": table, "suite": suite, "case": case, "d": 1, "realizations": M,
               "histories_per_realization": histories, "ours": {k: obs[k][0] for k in vals},
               "ours_sigma": {k: obs[k][1] for k in vals}, "paper": {k: vals[k][0] for k in vals}, "z": zs,
               "gpu_s": wall, "paper_t_tot_s": t_tot}
        if cls_histories > 0:
            c = paper_case(case, 1, suite, histories=cls_histories, seed=991000 + i)
            pc = make_problem(cls, c, True)
            cls.cls_set_stream(pc, stream)
            cls.cls_run(pc, cls_histories, c.seed)
            t, _, _ = cls.cls_read_tallies(pc, c.nbins)
            cls.cls_destroy_problem(pc)
            n = t.histories
            cobs = {"R": t.R, "T": t.T, "flux": t.total_flux, "Lk": 0.5 * (t.transmitted + t.reflected) / n}
            pcls = cls_rows[(suite, case, 1)]
            row["cls_error_pct"] = {k: 100.0 * (cobs[k] - obs[k][0]) / obs[k][0] for k in vals}
            row["paper_cls_error_pct"] = {k: 100.0 * (pcls[k][0] - vals[k][0]) / vals[k][0] for k in vals}
        out.append(row)
        msg = ", ".join(f"{k} z={zs[k]:+.2f}" for k in zs)
        if cls_histories > 0:
            msg += "; CLS error " + ", ".join(f"{k} {row['cls_error_pct'][k]:+.2f}% (paper "
                                              f"{row['paper_cls_error_pct'][k]:+.2f}%)" for k in zs)
        log(f"  {table} {suite:2s} {case} d=1 Ref, M={M}: {msg}; {wall:.2f} s (paper t_tot {t_tot:.3g} s)")
    return out


def run_quenched_leg(cls, torch, stream, perf_model, histories):
    """The quenched d = 1 reference kernel on one paper case (Table 3, case 1a,
    suite I slab, the paper's 1e4 realizations) at `histories` histories per
    realization: rate and roofline of the kernel (FP64)."""
    from paper_1708_00765_amd.inputs import paper_case
    s = paper_case("1a", 1, "I", histories=1, seed=880001)
    p = make_problem(cls, s, False)
    cls.cls_set_stream(p, stream)
    M = paper_realizations("I", "1a")
    cls.cls_run_quenched(p, 10, 10, s.seed + 1)                    # warm the code object
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cls.cls_run_quenched(p, M, histories, s.seed)
    g, _, _ = cls.cls_read_quenched(p, s.nbins)
    wall = time.perf_counter() - t0
    cls.cls_destroy_problem(p)
    n = M * histories
    slots = perf_model.quenched_slots(True, not s.collision, s.source == 0, n, g.flights, g.collisions, g.scatters)
    achieved = slots / (g.track_ms * 1e-3) / 1e12
    peak = perf_model.PEAK_SLOTS_PER_S / 1e12
    return {"workload": f"quenched d=1 slab, Table 3 case 1a suite I: {M} realizations x {histories} histories, "
                        f"{s.nbins} bins, track-length flux, FP64",
            "value": n / wall, "unit": "histories/s", "wall_ms": 1e3 * wall, "kernel_ms": g.track_ms,
            "flights_per_history": g.flights / n, "layers_per_realization": g.layers / M,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                         "frac": achieved / peak, "algorithmic_slots": slots}}


def _span(values):
    """One value, or the range of a mix (as "1e4 to 1e7")."""
    v = list(values)
    lo, hi = min(v), max(v)
    return f"{lo:g}" if lo == hi else f"{lo:g} to {hi:g}"


def run_ext2d_comparison(cls, torch, stream, steps):
    """The 256 uneven ext2d sets (1e4..1e7 histories, 100..1000 bins): one batched
    FP32 persistent launch per pass vs one plain FP64 launch per set, and the
    batched launch's VALU roofline (its kernel time from the library's events on
    the launch stream)."""
    from paper_1708_00765_amd import perf_model
    from paper_1708_00765_amd.inputs import workload
    specs = workload("ext2d_batched")
    total = sum(s.histories for s in specs)
    hist = [s.histories for s in specs]
    p32 = [make_problem(cls, s, fp32=True) for s in specs]
    p64 = [make_problem(cls, s, fp32=False) for s in specs]
    try:
        for p in p32 + p64:
            cls.cls_set_stream(p, stream)
        kernel_ms = []

        def time_batched():
            cls.cls_run_batch(p32, hist, [s.seed for s in specs])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ms = 0.0
            for k in range(steps):
                cls.cls_run_batch(p32, hist, [s.seed + k + 1 for s in specs])
                ms += cls.cls_read_tallies(p32[0], specs[0].nbins)[0].track_ms
            torch.cuda.synchronize()
            kernel_ms.append(ms / steps)
            return (time.perf_counter() - t0) / steps

        # default launch configuration, then the autotuner's choice for these sets
        # (timed before and after the tuned runs: the order is not what differs)
        w_default = time_batched()
        cfg, tuned_rate = cls.cls_autotune(p32, hist)
        w32 = time_batched()
        cls.cls_set_launch_config(0, 0, 0, 0)         # the FP64 plain runs use the defaults
        w_default = min(w_default, time_batched())
        for p, s in zip(p64[:8], specs[:8]):
            cls.cls_run(p, min(s.histories, 10000), s.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        full64 = None
        for k in range(steps):
            for p, s in zip(p64, specs):
                cls.cls_run(p, s.histories, s.seed + k + 1)
            if k == 0:
                full64 = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(p64, specs)]
        torch.cuda.synchronize()
        w64 = (time.perf_counter() - t0) / steps
        # the FP32 batched form on the seeds of the first FP64 pass (same streams)
        cls.cls_run_batch(p32, hist, [s.seed + 1 for s in specs])
        full32 = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(p32, specs)]
    finally:
        for p in p32 + p64:
            cls.cls_destroy_problem(p)
    tallies = [f[0] for f in full32]
    slots = perf_model.algorithmic_slots("ext2d", total, sum(t.flights for t in tallies),
                                         sum(t.scatters for t in tallies),
                                         sum(t.lateral_reflections for t in tallies), fp32=True, track=True)
    k_ms = kernel_ms[1]                       # the tuned configuration's passes
    achieved = slots / (k_ms * 1e-3) / 1e12
    peak = perf_model.PEAK_SLOTS_PER_S / 1e12
    return {"sets": len(specs), "histories": total, "fp32_batched_value": total / w32,
            "fp64_plain_value": total / w64, "ratio": w64 / w32, "fp32_batched_ms": 1e3 * w32,
            "fp64_plain_ms": 1e3 * w64, "unit": "histories/s", "autotuned_config": cfg,
            "fp32_batched_default_config_value": total / w_default,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                         "frac": achieved / peak, "kernel_ms": k_ms, "algorithmic_slots_per_launch": slots,
                         "flights_per_history": sum(t.flights for t in tallies) / total},
            "fp32_vs_fp64_same_streams": fp32_acceptance(full32, full64)}


def _server_line(cls, srv, label):
    st = cls.cls_server_get_stats(srv)
    return (f"{label}: submitted {st['submitted']}, completed {st['completed']}, failed {st['failed']}, "
            f"pending {st['pending']}, active {st['active']}, rounds {st['rounds']}")


def _wait_all(cls, srv, tickets, label, limit_s=60.0):
    """Wait for every ticket, logging progress every 10 s; a request that is not
    done `limit_s` after the previous completion ends the leg with an error."""
    last = time.perf_counter()
    for tk in tickets:
        while not cls.cls_server_wait(srv, tk, 10.0):
            log(_server_line(cls, srv, label + " (waiting)"))
            if time.perf_counter() - last > limit_s:
                raise RuntimeError(f"{label}: request {tk} not done {limit_s:.0f} s after the previous one; "
                                   + _server_line(cls, srv, "server"))
        last = time.perf_counter()


def _latency_stages(infos):
    """p50 / p99 in ms of each stage of a served request: submission to its first
    chunk published, to the completion signal seen by the worker, to the finalize
    launch, to the result on the host."""
    import numpy as np
    keys = ("submit_s", "publish_s", "signal_s", "finalize_s", "done_s")
    out = {}
    for a, b in zip(keys, keys[1:]):
        d = np.array([i[b] - i[a] for i in infos if i[a] >= 0 and i[b] >= 0]) * 1e3
        if len(d):
            out[f"{a[:-2]}_to_{b[:-2]}"] = {"p50": float(np.percentile(d, 50)), "p99": float(np.percentile(d, 99))}
    return out


# Served requests kept for the comparison with the FP64 oracle (in the CPU
# baseline leg): the first ones of at most this many histories.
SERVED_ORACLE_SAMPLE = 16
SERVED_ORACLE_MAX_HISTORIES = 200_000


def run_served(cls, seconds, rate):
    """Submit the served workload's Poisson stream in real time; latency is
    arrival to results on the host, measured by the server's clock. Also keeps
    the results of a bounded sample of small requests (key `_oracle_sample`, not
    reported) for the comparison with the oracle."""
    from paper_1708_00765_amd.inputs import served_requests
    import numpy as np
    reqs = served_requests(rate_hz=rate, duration_s=seconds)
    srv = cls.cls_server_create()
    live = []
    t0 = time.perf_counter()
    next_log = 10.0
    log(f"served: {len(reqs)} requests over {seconds:g} s")
    try:
        for t_arr, s in reqs:
            delay = t0 + t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            if t_arr >= next_log:
                log(_server_line(cls, srv, f"served at {t_arr:.0f} s"))
                next_log += 10.0
            p = make_problem(cls, s, fp32=True)
            live.append((cls.cls_server_submit(srv, p, s.histories, s.seed), p, s))
        _wait_all(cls, srv, [tk for tk, _, _ in live], "served")
        infos = [cls.cls_server_request_info(srv, tk) for tk, _, _ in live]
        stats = cls.cls_server_get_stats(srv)
        sample = [(s, cls.cls_read_tallies(p, s.nbins)) for _, p, s in live
                  if s.histories <= SERVED_ORACLE_MAX_HISTORIES][:SERVED_ORACLE_SAMPLE]
    finally:
        cls.cls_server_destroy(srv)
        for _, p, _ in live:
            cls.cls_destroy_problem(p)
    lat = np.array([i["done_s"] - i["submit_s"] for i in infos]) * 1e3
    stages = _latency_stages(infos)
    first = min(i["submit_s"] for i in infos)
    last = max(i["done_s"] for i in infos)
    hist = sum(i["histories"] for i in infos)
    return {"requests": len(reqs), "completed": stats["completed"], "failed": stats["failed"],
            "offered_rate_hz": rate, "seconds": seconds,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "histories": hist, "histories_per_s": hist / (last - first),
            "offered_histories_per_s": hist / seconds, "rounds": stats["rounds"],
            "wave_idle_share": stats["wave_idle_share"],
            "hbm_peak_bytes": stats["hbm_peak"], "latency_stages_ms": stages, "_oracle_sample": sample,
            "workload": "served: d uniform in {1 (rod, collision flux), 2 (ext2d), 3 (cube3d)}, "
                        "histories log-uniform in [1e4, 1e8], 10-1000 bins, FP32 tracking"}


def run_served_saturated(cls, rate, seconds):
    """The served request mix at saturation: every request of `seconds` of a
    Poisson stream at `rate` submitted at once; throughput over the makespan
    (first submission to last result on the host) and the algorithmic VALU
    roofline fraction of the served form."""
    from paper_1708_00765_amd import perf_model
    from paper_1708_00765_amd.inputs import served_requests
    specs = [s for _, s in served_requests(rate_hz=rate, duration_s=seconds)]
    probs = [make_problem(cls, s, fp32=True) for s in specs]
    srv = cls.cls_server_create()
    try:
        tickets = [cls.cls_server_submit(srv, p, s.histories, s.seed) for p, s in zip(probs, specs)]
        _wait_all(cls, srv, tickets, "served at saturation")
        infos = [cls.cls_server_request_info(srv, tk) for tk in tickets]
        stats = cls.cls_server_get_stats(srv)
    finally:
        cls.cls_server_destroy(srv)
    try:
        slots = 0.0
        flights = 0
        for p, s in zip(probs, specs):
            t, _, _ = cls.cls_read_tallies(p, s.nbins)
            flights += t.flights
            slots += perf_model.algorithmic_slots(s.geom_name, t.histories, t.flights, t.scatters,
                                                  t.lateral_reflections, fp32=True, track=not s.collision)
    finally:
        for p in probs:
            cls.cls_destroy_problem(p)
    span = max(i["done_s"] for i in infos) - min(i["submit_s"] for i in infos)
    hist = sum(s.histories for s in specs)
    achieved = slots / span / 1e12
    peak = perf_model.PEAK_SLOTS_PER_S / 1e12
    return {"requests": len(specs), "completed": stats["completed"], "failed": stats["failed"],
            "histories": hist, "flights": flights, "seconds": span, "value": hist / span, "unit": "histories/s",
            "rounds": stats["rounds"], "wave_idle_share": stats["wave_idle_share"],
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                         "frac": achieved / peak, "algorithmic_slots": slots},
            "workload": f"served mix (as the Poisson stream), the {len(specs)} requests of {seconds:g} s at "
                        f"{rate:g} requests/s submitted at once"}


def physical_cpu():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = "", set()
    phys = core = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and not model:
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None and core is not None:
                cores.add((phys, core))
                phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, (len(cores) or None)


def run_form(cls, torch, stream, perf_model, specs, steps, warmup, fp64_steps, label, tune=False, max_chunk=0):
    """One workload: `steps` timed batched FP32 launches (after `warmup`), then the
    plain FP64 one-problem-per-launch runs, the first of them on the seeds of the last
    timed FP32 step (common random numbers: the acceptance rule of the FP32 form).
    With `tune`, the FP32 launches use the autotuner's launch configuration for these
    sets, and the default configuration is timed as well for comparison."""
    total_hist = sum(s.histories for s in specs)
    geom = specs[0].geom_name
    probs = [make_problem(cls, s, fp32=True) for s in specs]
    for p in probs:
        cls.cls_set_stream(p, stream)
    log(f"{label}: fp32 batched, {len(specs)} sets x {_span(s.histories for s in specs)} histories, "
        f"{warmup} warmup + {steps} steps")
    tuning = None
    try:
        if max_chunk > 0:
            cls.cls_set_launch_config(0, 0, max_chunk, 0)
            tuning = {"max_chunk": max_chunk}
        elif tune:
            cls.cls_set_launch_config(0, 0, 0, 0)
            d_steps = max(1, min(steps, 3))
            d_wall, d_ms, _ = run_batch_steps(cls, torch, probs, specs, d_steps, 1, 1000)
            t0 = time.perf_counter()
            cfg, tuned_rate = cls.cls_autotune(probs, [s.histories for s in specs])
            tuning = {"autotuned_config": cfg, "autotune_seconds": time.perf_counter() - t0,
                      "default_config_value": total_hist * d_steps / d_wall,
                      "default_config_kernel_ms": d_ms / d_steps, "default_config_steps": d_steps}
            log(f"  autotuned {cfg} in {tuning['autotune_seconds']:.1f} s; default configuration "
                f"{tuning['default_config_value']:.4g} hist/s ({d_steps} steps)")
        wall, track_ms, full32 = run_batch_steps(cls, torch, probs, specs, steps, warmup, 0)
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)
        for p in probs:
            cls.cls_destroy_problem(p)
    tallies = [f[0] for f in full32]
    last_step = warmup + steps - 1
    value = total_hist * steps / wall
    flights = sum(t.flights for t in tallies)
    collisions = sum(t.collisions for t in tallies)
    scatters = sum(t.scatters for t in tallies)
    lateral = sum(t.lateral_reflections for t in tallies)
    kernel_ms = track_ms / steps
    slots = perf_model.algorithmic_slots(geom, total_hist, flights, scatters, lateral, fp32=True,
                                         track=not specs[0].collision)
    achieved = slots / (kernel_ms * 1e-3) / 1e12
    peak = perf_model.PEAK_SLOTS_PER_S / 1e12
    out = {"value": value, "unit": "histories/s", "ms_per_step": 1e3 * wall / steps, "kernel_ms": kernel_ms,
           "launch_config": tuning if tuning else "default",
           "collisions_per_s": collisions * steps / wall, "flights_per_s": flights * steps / wall,
           "flights_per_history": flights / total_hist, "histories_per_step": total_hist,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                        "frac": achieved / peak, "kernel_ms": kernel_ms, "algorithmic_slots_per_launch": slots}}
    log(f"  {out['ms_per_step']:.1f} ms/step, kernel {kernel_ms:.1f} ms, {value:.4g} hist/s, "
        f"{flights / total_hist:.2f} flights/hist, {achieved:.2f}/{peak:.2f} Tslot/s (frac {achieved / peak:.3f})")
    if fp64_steps > 0:
        probs64 = [make_problem(cls, s, fp32=False) for s in specs]
        try:
            for p in probs64:
                cls.cls_set_stream(p, stream)
            for p, s in zip(probs64, specs):           # warm the FP64 code object
                cls.cls_run(p, min(s.histories, 100_000), s.seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k64 = 0.0
            full64 = None
            for k in range(fp64_steps):
                for p, s in zip(probs64, specs):
                    cls.cls_run(p, s.histories, (s.seed + 0x9E3779B97F4A7C15 * (last_step + k)) & (2**64 - 1))
                    k64 += cls.cls_read_tallies(p, s.nbins)[0].track_ms
                if k == 0:
                    full64 = [cls.cls_read_tallies(p, s.nbins) for p, s in zip(probs64, specs)]
            torch.cuda.synchronize()
            w64 = time.perf_counter() - t0
        finally:
            for p in probs64:
                cls.cls_destroy_problem(p)
        v64 = total_hist * fp64_steps / w64
        out["fp64_plain"] = {"value": v64, "unit": "histories/s", "ms_per_step": 1e3 * w64 / fp64_steps,
                             "kernel_ms_per_step": k64 / fp64_steps, "launches_per_step": len(specs)}
        out["speedup_vs_fp64_plain"] = value / v64
        acc = fp32_acceptance(full32, full64)
        out["fp32_vs_fp64_same_streams"] = acc
        log(f"  fp64 plain: {1e3 * w64 / fp64_steps:.1f} ms/step, {v64:.4g} hist/s, FP32/FP64 {value / v64:.2f}x; "
            f"FP32 vs FP64 (same streams): scalars {acc['max_rel_scalar']:.2e}, profile "
            f"{acc['max_rel_profile_l2']:.2e}, worst bin {acc['max_bin_deviation_over_allowance']:.3f} of its "
            f"allowance, violations {acc['violations']} -> {'passes' if acc['passes'] else 'FAILS'}")
    return out, full32


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stress3d")
    ap.add_argument("--histories", type=int, default=0, help="override histories per set")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed passes of the FP64 plain leg (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="oracle sample budget (0 = skip)")
    ap.add_argument("--max-chunk", type=int, default=0,
                    help="histories per work chunk of the main workload's FP32 launches "
                         "(0: the launch configuration's; implies --autotune 0)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: the main workload's FP32 launches use the autotuned configuration "
                         "(the default configuration is timed as well); 0: default configuration")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--cube3d-steps", type=int, default=3,
                    help="timed steps of the cube3d_track leg (8 sets x 1e8, 200 bins; 0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served Poisson request stream (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="request arrival rate (1/s)")
    ap.add_argument("--saturate-seconds", type=float, default=2.0,
                    help="served mix at saturation: requests of this many seconds at 600/s, "
                         "submitted at once (0 = skip)")
    ap.add_argument("--ext2d-steps", type=int, default=2,
                    help="timed passes of the 256-set ext2d comparison (0 = skip)")
    ap.add_argument("--paper-rows", type=float, default=0,
                    help="histories per row for the 54 CLS rows of Tables 3-8 (0 = skip; the paper used 1e9)")
    ap.add_argument("--paper-precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--paper-ref-rows", type=float, default=0,
                    help="histories per realization for the 18 d = 1 quenched reference rows of Tables 3-8 "
                         "(0 = skip; the paper used 1e6), at the paper's realization counts")
    ap.add_argument("--paper-ref-cls", type=float, default=1e9,
                    help="histories of the CLS run compared with each reference row (0 = skip)")
    ap.add_argument("--quenched-histories", type=float, default=1e5,
                    help="histories per realization of the quenched d = 1 kernel leg (0 = skip)")
    ap.add_argument("--paper-out", default="", help="write the per-row results of --paper-rows to this JSON file")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(CLS histories are independent: a multi-GPU run would shard history ranges "
              "and all-reduce the tallies, which this library does not implement).", flush=True)
        return 2

    import torch

    from paper_1708_00765_amd import cls, perf_model
    from paper_1708_00765_amd.inputs import workload

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    specs = workload(args.workload, histories=args.histories or None)
    total_hist = sum(s.histories for s in specs)
    geom = specs[0].geom_name

    # ---- the main workload: FP32 batched (timed steps) vs FP64 plain ----------
    main_leg, full32 = run_form(cls, torch, stream, perf_model, specs, args.steps, args.warmup, args.fp64_steps,
                                args.workload, tune=bool(args.autotune) and args.max_chunk <= 0,
                                max_chunk=args.max_chunk)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # ---- cube3d_track: 8 sets x 1e8, 200 bins ----------------------------------
    cube = None
    if args.cube3d_steps > 0 and args.workload != "cube3d_track":
        cube, _ = run_form(cls, torch, stream, perf_model, workload("cube3d_track"), args.cube3d_steps, 1,
                           1, "cube3d_track")
        cube["workload"] = ("cube3d_track: 8 sets x 1e8 histories, d=3 cube, L=10, 200 x-bins, track-length flux, "
                            "Sigma_i log-uniform [0.02, 2], c_i uniform [0, 1], Lambda_i log-uniform [0.1, 10]")
        cube["traffic"] = measured_traffic("cube3d_track")

    # ---- 256 uneven ext2d sets: one batched FP32 launch vs one FP64 launch per set --
    ext2d = None
    if args.ext2d_steps > 0:
        ext2d = run_ext2d_comparison(cls, torch, stream, args.ext2d_steps)
        log(f"ext2d 256 sets: fp32 batched {ext2d['fp32_batched_value']:.4g} hist/s (autotuned "
            f"{ext2d['autotuned_config']}; default configuration "
            f"{ext2d['fp32_batched_default_config_value']:.4g}), fp64 plain "
            f"{ext2d['fp64_plain_value']:.4g} hist/s, ratio {ext2d['ratio']:.2f}, "
            f"roofline frac {ext2d['roofline']['frac']:.3f}")

    # ---- quenched d = 1 reference kernel -------------------------------------------
    quenched = None
    if args.quenched_histories > 0:
        quenched = run_quenched_leg(cls, torch, stream, perf_model, int(args.quenched_histories))
        log(f"quenched d=1: {quenched['value']:.4g} hist/s, kernel {quenched['kernel_ms']:.1f} ms, "
            f"{quenched['flights_per_history']:.2f} flights/hist, roofline frac {quenched['roofline']['frac']:.3f}")

    # ---- served: Poisson request stream through the continuous-batching server --
    served = None
    if args.serve_seconds > 0:
        served = run_served(cls, args.serve_seconds, args.serve_rate)
        log(f"served: {served['completed']} requests, p50 {served['p50_ms']:.1f} ms, "
            f"p99 {served['p99_ms']:.1f} ms, {served['histories_per_s']:.4g} hist/s; stages (p50/p99 ms) "
            + ", ".join(f"{k} {v['p50']:.2f}/{v['p99']:.2f}" for k, v in served["latency_stages_ms"].items()))
    served_sat = None
    if args.saturate_seconds > 0:
        served_sat = run_served_saturated(cls, 600.0, args.saturate_seconds)
        log(f"served at saturation: {served_sat['requests']} requests, {served_sat['value']:.4g} hist/s, "
            f"roofline frac {served_sat['roofline']['frac']:.3f}")

    # ---- the paper's own benchmark rows ---------------------------------------
    paper = None
    if args.paper_rows > 0:
        log(f"paper rows: 54 CLS rows of Tables 3-8, {args.paper_rows:.3g} histories each, {args.paper_precision}")
        rows = run_paper_rows(cls, torch, stream, int(args.paper_rows), args.paper_precision == "fp32")
        zmax = max(abs(v) for r in rows for v in r["z"].values())
        paper = {"rows": len(rows), "histories_per_row": int(args.paper_rows), "precision": args.paper_precision,
                 "max_abs_z": zmax, "beyond_4_sigma": sum(1 for r in rows for v in r["z"].values() if abs(v) >= 4),
                 "gpu_seconds": sum(r["gpu_s"] for r in rows),
                 "paper_t_tot_seconds": sum(r["paper_t_tot_s"] for r in rows)}
        log(f"paper rows: max |z| {zmax:.2f}, {paper['beyond_4_sigma']} beyond 4 sigma, GPU "
            f"{paper['gpu_seconds']:.1f} s vs paper t_tot {paper['paper_t_tot_seconds']:.3g} s")
        if args.paper_out:
            with open(args.paper_out, "w") as f:
                json.dump({"summary": paper, "rows": rows}, f, indent=1)

    # ---- the paper's d = 1 quenched reference rows ------------------------------
    paper_ref = None
    if args.paper_ref_rows > 0:
        log(f"paper reference rows: 18 d = 1 Ref rows of Tables 3-8, {args.paper_ref_rows:.3g} histories "
            f"per realization, FP64")
        rows = run_paper_ref_rows(cls, torch, stream, int(args.paper_ref_rows), int(args.paper_ref_cls))
        zmax = max(abs(v) for r in rows for v in r["z"].values())
        paper_ref = {"rows": len(rows), "histories_per_realization": int(args.paper_ref_rows),
                     "max_abs_z": zmax,
                     "beyond_4_sigma": sum(1 for r in rows for v in r["z"].values() if abs(v) >= 4),
                     "gpu_seconds": sum(r["gpu_s"] for r in rows),
                     "paper_t_tot_seconds": sum(r["paper_t_tot_s"] for r in rows)}
        log(f"paper reference rows: max |z| {zmax:.2f}, {paper_ref['beyond_4_sigma']} beyond 4 sigma, GPU "
            f"{paper_ref['gpu_seconds']:.1f} s vs paper t_tot {paper_ref['paper_t_tot_seconds']:.3g} s")
        if args.paper_out:
            base, ext = os.path.splitext(args.paper_out)
            with open(base + "_ref" + (ext or ".json"), "w") as f:
                json.dump({"summary": paper_ref, "rows": rows}, f, indent=1)

    # ---- CPU oracle on a bounded sample of the main workload -------------------
    cpu = None
    oracle_vs = None
    if args.cpu_seconds > 0:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from oracle import oracle
        from helpers import run_oracle
        # calibrate on a sample large enough that thread start-up does not dominate
        per = 2000
        while True:
            t0 = time.perf_counter()
            for s in specs:
                run_oracle(s, histories=per, seed=s.seed + 7)
            cal = time.perf_counter() - t0
            if cal > 0.05 * args.cpu_seconds or per >= 10**8:
                break
            per *= 4
        n_each = max(per, int(per * args.cpu_seconds / max(cal, 1e-6)))
        t0 = time.perf_counter()
        coll = 0
        orc = []
        for s in specs:
            r = run_oracle(s, histories=n_each, seed=s.seed + 11)
            coll += r.collisions
            orc.append(r)
        tc = time.perf_counter() - t0
        # one thread on a sample a tenth of the size (histories are independent,
        # so rates extrapolate linearly)
        n_one = max(100, n_each // (10 * max(1, oracle.max_threads())))
        t1 = time.perf_counter()
        for s in specs:
            run_oracle(s, histories=n_one, seed=s.seed + 13, threads=1)
        t1 = time.perf_counter() - t1
        cpu_model, phys = physical_cpu()
        cpu = {"value": n_each * len(specs) / tc, "unit": "histories/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"the {len(specs)} {args.workload} parameter sets x {n_each} histories each "
                         f"({tc:.1f} s, FP64, OpenMP over 4096-history chunks, {oracle.max_threads()} threads)",
               "collisions_per_s": coll / tc,
               "single_thread_value": n_one * len(specs) / t1,
               "single_thread_sample": f"{len(specs)} sets x {n_one} histories ({t1:.1f} s, 1 thread)",
               "cpu_model": cpu_model, "physical_cores": phys, "logical_cpus": os.cpu_count()}
        log(f"cpu oracle: {cpu['value']:.4g} hist/s on {cpu['cores']} threads "
            f"({cpu['single_thread_value']:.4g} on 1 thread; {cpu_model}, {phys} physical cores)")
        # the same oracle runs are the FP64 reference of the FP32 results (independent streams)
        oracle_vs = oracle_agreement(full32, orc)
        log(f"fp32 batched vs the FP64 oracle ({n_each} histories per set): max |z| {oracle_vs['max_abs_z_scalars']:.2f}, "
            f"bins beyond 4 sigma {oracle_vs['bins_beyond_4_sigma']} of {oracle_vs['bins']} "
            f"(allowed {oracle_vs['bins_beyond_4_sigma_allowed']})")
        # served requests (FP32) against oracle runs of the same requests on independent streams
        if served and served.get("_oracle_sample"):
            sample = served["_oracle_sample"]
            orc_s = [run_oracle(s, seed=s.seed ^ 0x5DEECE66D) for s, _ in sample]
            sv = oracle_agreement([t for _, t in sample], orc_s)
            sv.pop("oracle_histories_per_set", None)
            sv["requests"] = len(sample)
            sv["sample"] = (f"the first {len(sample)} served requests of at most {SERVED_ORACLE_MAX_HISTORIES} "
                            "histories, each against the FP64 oracle on independent streams")
            served["fp32_vs_oracle"] = sv
            log(f"served vs the FP64 oracle ({len(sample)} requests): max |z| {sv['max_abs_z_scalars']:.2f}, "
                f"bins beyond 4 sigma {sv['bins_beyond_4_sigma']} of {sv['bins']} "
                f"(allowed {sv['bins_beyond_4_sigma_allowed']})")

    traffic = measured_traffic(args.workload) if not args.histories else None
    kernel_ms = main_leg["kernel_ms"]
    roof = dict(main_leg["roofline"])
    roof.update({"traffic": traffic,
                 "traffic_unit": "HBM bytes per tracking launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                 "traffic_gb_per_s": (traffic / (kernel_ms * 1e-3) / 1e9) if traffic else None})
    line = {
        "metric": "histories/s on 1 MI355X, FP32-batched vs plain FP64 CLS; p50/p99 req latency",
        "value": main_leg["value"],
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {len(specs)} sets x {_span(s.histories for s in specs)} histories, "
                               f"d={specs[0].d} ({geom}), L={specs[0].L:g}, {_span(s.nbins for s in specs)} x-bins, "
                               f"{'collision' if specs[0].collision else 'track-length'} flux, "
                               "FP32 tracking with FP64 positions and tallies, one batched persistent launch per step",
                   "sets": len(specs), "histories_per_step": total_hist},
        "collisions_per_s": main_leg["collisions_per_s"],
        "flights_per_s": main_leg["flights_per_s"],
        "flights_per_history": main_leg["flights_per_history"],
        "launch_config": main_leg["launch_config"],
        "fp64_plain": main_leg.get("fp64_plain"),
        "speedup_vs_fp64_plain": main_leg.get("speedup_vs_fp64_plain"),
        "fp32_vs_fp64_same_streams": main_leg.get("fp32_vs_fp64_same_streams"),
        "fp32_vs_oracle": oracle_vs,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cube3d_track": cube,
        "served": {k: v for k, v in served.items() if not k.startswith("_")} if served else None,
        "served_saturated": served_sat,
        "ext2d_batched_vs_fp64_plain": ext2d,
        "paper_rows": paper,
        "paper_reference_rows": paper_ref,
        "quenched_d1": quenched,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
