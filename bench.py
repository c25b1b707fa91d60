#!/usr/bin/env python3
"""Throughput of Chord Length Sampling (Algorithm A, arXiv 1708.00765 Section 4)
on one MI355X.

Default workload (cube3d_track): d=3 cube of side 10, vacuum x-faces, mirroring
lateral faces, cosine-weighted incidence on x=0; 8 seeded parameter sets
(Sigma_i log-uniform in [0.02, 2], c_i uniform in [0, 1], Lambda_i log-uniform
in [0.1, 10]); 1e8 histories per set; 200 x-bins with the track-length
estimator. A step runs all 8 sets in one batched persistent launch with FP32
flight arithmetic and FP64 tallies, then finalizes and copies the results back.

Also reported: the plain FP64 one-problem-per-launch rate on the same sets, the
roofline of the tracking kernel (VALU issue slots, see perf_model.py) and the
FP64 CPU oracle on a bounded sample of the same sets.

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
    tallies = [cls.cls_read_tallies(p, s.nbins)[0] for p, s in zip(probs, specs)]
    return wall, track_ms, tallies


def run_ext2d_comparison(cls, torch, stream, steps):
    """The 256 uneven ext2d sets (1e4..1e7 histories, 100..1000 bins): one batched
    FP32 persistent launch per pass vs one plain FP64 launch per set."""
    from paper_1708_00765_amd.inputs import workload
    specs = workload("ext2d_batched")
    total = sum(s.histories for s in specs)
    hist = [s.histories for s in specs]
    p32 = [make_problem(cls, s, fp32=True) for s in specs]
    p64 = [make_problem(cls, s, fp32=False) for s in specs]
    try:
        for p in p32 + p64:
            cls.cls_set_stream(p, stream)
        cls.cls_run_batch(p32, hist, [s.seed for s in specs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            cls.cls_run_batch(p32, hist, [s.seed + k + 1 for s in specs])
        torch.cuda.synchronize()
        w32 = (time.perf_counter() - t0) / steps
        for p, s in zip(p64[:8], specs[:8]):
            cls.cls_run(p, min(s.histories, 10000), s.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            for p, s in zip(p64, specs):
                cls.cls_run(p, s.histories, s.seed + k + 1)
        torch.cuda.synchronize()
        w64 = (time.perf_counter() - t0) / steps
    finally:
        for p in p32 + p64:
            cls.cls_destroy_problem(p)
    return {"sets": len(specs), "histories": total, "fp32_batched_value": total / w32,
            "fp64_plain_value": total / w64, "ratio": w64 / w32, "fp32_batched_ms": 1e3 * w32,
            "fp64_plain_ms": 1e3 * w64, "unit": "histories/s"}


def run_served(cls, seconds, rate):
    """Submit the served workload's Poisson stream in real time; latency is
    arrival to results on the host, measured by the server's clock."""
    from paper_1708_00765_amd.inputs import served_requests
    import numpy as np
    reqs = served_requests(rate_hz=rate, duration_s=seconds)
    srv = cls.cls_server_create()
    live = []
    t0 = time.perf_counter()
    try:
        for t_arr, s in reqs:
            delay = t0 + t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            p = make_problem(cls, s, fp32=True)
            live.append((cls.cls_server_submit(srv, p, s.histories, s.seed), p, s))
        infos = []
        for tk, p, s in live:
            cls.cls_server_wait(srv, tk, 600.0)
            infos.append(cls.cls_server_request_info(srv, tk))
        stats = cls.cls_server_get_stats(srv)
    finally:
        cls.cls_server_destroy(srv)
        for _, p, _ in live:
            cls.cls_destroy_problem(p)
    lat = np.array([i["done_s"] - i["submit_s"] for i in infos]) * 1e3
    first = min(i["submit_s"] for i in infos)
    last = max(i["done_s"] for i in infos)
    hist = sum(i["histories"] for i in infos)
    return {"requests": len(reqs), "completed": stats["completed"], "failed": stats["failed"],
            "offered_rate_hz": rate, "seconds": seconds,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "histories": hist, "histories_per_s": hist / (last - first),
            "offered_histories_per_s": hist / seconds, "rounds": stats["rounds"],
            "hbm_peak_bytes": stats["hbm_peak"],
            "workload": "served: d uniform in {1 (rod, collision flux), 2 (ext2d), 3 (cube3d)}, "
                        "histories log-uniform in [1e4, 1e8], 10-1000 bins, FP32 tracking"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube3d_track")
    ap.add_argument("--histories", type=int, default=0, help="override histories per set")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed passes of the FP64 plain leg (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=15.0,
                    help="length of the served Poisson request stream (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="request arrival rate (1/s)")
    ap.add_argument("--ext2d-steps", type=int, default=2,
                    help="timed passes of the 256-set ext2d comparison (0 = skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(CLS histories are independent: a multi-GPU run would shard history ranges "
              "and all-reduce the tallies, which this build does not implement).", flush=True)
        return 2

    import torch

    from paper_1708_00765_amd import cls, perf_model
    from paper_1708_00765_amd.inputs import workload

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    specs = workload(args.workload, histories=args.histories or None)
    total_hist = sum(s.histories for s in specs)
    geom = specs[0].geom_name

    # ---- FP32 batched: the timed steps ----------------------------------
    probs = [make_problem(cls, s, fp32=True) for s in specs]
    for p in probs:
        cls.cls_set_stream(p, stream)
    log(f"fp32 batched: {len(specs)} sets x {specs[0].histories:.3g} histories, "
        f"{args.warmup} warmup + {args.steps} steps")
    wall, track_ms, tallies = run_batch_steps(cls, torch, probs, specs, args.steps, args.warmup, 0)
    ms_per_step = 1e3 * wall / args.steps
    value = total_hist * args.steps / wall
    flights = sum(t.flights for t in tallies)
    collisions = sum(t.collisions for t in tallies)
    scatters = sum(t.scatters for t in tallies)
    lateral = sum(t.lateral_reflections for t in tallies)
    kernel_ms = track_ms / args.steps
    slots = perf_model.algorithmic_slots(geom, total_hist, flights, scatters, lateral, fp32=True,
                                         track=not specs[0].collision)
    achieved = slots / (kernel_ms * 1e-3) / 1e12
    peak = perf_model.PEAK_SLOTS_PER_S / 1e12
    log(f"  {ms_per_step:.1f} ms/step, kernel {kernel_ms:.1f} ms, {value:.4g} hist/s, "
        f"{flights / total_hist:.2f} flights/hist, {achieved:.2f}/{peak:.2f} Tslot/s")
    for p in probs:
        cls.cls_destroy_problem(p)

    # ---- FP64 plain: one problem per launch ----------------------------------
    fp64 = None
    if args.fp64_steps > 0:
        probs64 = [make_problem(cls, s, fp32=False) for s in specs]
        for p in probs64:
            cls.cls_set_stream(p, stream)
        for p, s in zip(probs64, specs):           # warm the FP64 code object
            cls.cls_run(p, min(s.histories, 100_000), s.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k64 = 0.0
        for k in range(args.fp64_steps):
            for p, s in zip(probs64, specs):
                cls.cls_run(p, s.histories, (s.seed + 0x9E3779B97F4A7C15 * (k + 1)) & (2**64 - 1))
                k64 += cls.cls_read_tallies(p, s.nbins)[0].track_ms
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t0
        v64 = total_hist * args.fp64_steps / w64
        fp64 = {"value": v64, "unit": "histories/s", "ms_per_step": 1e3 * w64 / args.fp64_steps,
                "kernel_ms_per_step": k64 / args.fp64_steps, "launches_per_step": len(specs)}
        log(f"fp64 plain: {fp64['ms_per_step']:.1f} ms/step, {v64:.4g} hist/s")
        for p in probs64:
            cls.cls_destroy_problem(p)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # ---- 256 uneven ext2d sets: one batched FP32 launch vs one FP64 launch per set --
    ext2d = None
    if args.ext2d_steps > 0:
        ext2d = run_ext2d_comparison(cls, torch, stream, args.ext2d_steps)
        log(f"ext2d 256 sets: fp32 batched {ext2d['fp32_batched_value']:.4g} hist/s, fp64 plain "
            f"{ext2d['fp64_plain_value']:.4g} hist/s, ratio {ext2d['ratio']:.2f}")

    # ---- served: Poisson request stream through the continuous-batching server --
    served = None
    if args.serve_seconds > 0:
        served = run_served(cls, args.serve_seconds, args.serve_rate)
        log(f"served: {served['completed']} requests, p50 {served['p50_ms']:.1f} ms, "
            f"p99 {served['p99_ms']:.1f} ms, {served['histories_per_s']:.4g} hist/s")

    # ---- CPU oracle on a bounded sample ---------------------------------------
    cpu = None
    if args.cpu_seconds > 0:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from oracle import oracle
        from helpers import run_oracle
        # calibrate on a sample large enough that thread start-up does not dominate
        per = 20000
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
        for s in specs:
            run_oracle(s, histories=n_each, seed=s.seed + 11)
        tc = time.perf_counter() - t0
        cpu = {"value": n_each * len(specs) / tc, "unit": "histories/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"the {len(specs)} {args.workload} parameter sets x {n_each} histories each "
                         f"({tc:.1f} s, FP64, OpenMP over 4096-history chunks)"}
        log(f"cpu oracle: {cpu['value']:.4g} hist/s on {cpu['cores']} threads")

    line = {
        "metric": "histories/s on 1 MI355X, FP32-batched vs plain FP64 CLS; p50/p99 req latency",
        "value": value,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {len(specs)} sets x {specs[0].histories:g} histories, "
                               f"d={specs[0].d} ({geom}), L={specs[0].L:g}, {specs[0].nbins} x-bins, "
                               f"{'collision' if specs[0].collision else 'track-length'} flux, "
                               "FP32 tracking with FP64 tallies, one batched persistent launch per step",
                   "sets": len(specs), "histories_per_step": total_hist},
        "collisions_per_s": collisions * args.steps / wall,
        "flights_per_s": flights * args.steps / wall,
        "flights_per_history": flights / total_hist,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel_ms": kernel_ms, "algorithmic_slots_per_launch": slots},
        "cpu_baseline": cpu,
        "served": served,
        "ext2d_batched_vs_fp64_plain": ext2d,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
