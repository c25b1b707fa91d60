"""The allocation-free entry point (cls_run_static) against cls_run: two calls in a
row on one device, the second with a smaller problem (fewer histories and bins),
each equal to the same run through cls_run. With every chunk its own error batch
(chunk_batches = 1) the records are equal (integer tallies bitwise, FP64 sums to
summation order); with the default gathering of chunks into batches, whose
composition follows the order in which waves take chunks, the counts, means and
per-history errors are equal and the per-bin flux errors agree statistically.
Sizes beyond the static workspace are refused. All GPU calls go through the C ABI;
the result buffer is caller-owned device memory (a torch tensor)."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import gpu_problem, tallies_dict
from paper_1708_00765_amd.inputs import Spec

pytestmark = pytest.mark.gpu

COUNTS = ("histories", "transmitted", "reflected", "absorbed", "capped", "flights", "collisions", "scatters",
          "interface_crossings", "lateral_reflections")


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1708_00765_amd import cls
    cls.cls_set_launch_config(0, 0, 0, 0)
    return torch, cls


def _static_run(torch, cls, s, fp32):
    p = gpu_problem(s, fp32=fp32)
    try:
        nbytes = cls.record_bytes(s.nbins)
        buf = torch.zeros(nbytes // 8, dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        cls.cls_run_static(p, s.histories, s.seed, stream.cuda_stream, buf.data_ptr(), nbytes)
        torch.cuda.synchronize()
        rec, flux, fsig = cls.decode_record(buf.cpu().numpy().view(np.uint64), s.nbins)
    finally:
        cls.cls_destroy_problem(p)
    return rec, flux, fsig


def _plain_run(cls, s, fp32):
    p = gpu_problem(s, fp32=fp32)
    try:
        cls.cls_run(p, s.histories, s.seed)
        t, flux, fsig = cls.cls_read_tallies(p, s.nbins)
    finally:
        cls.cls_destroy_problem(p)
    return tallies_dict(t), flux, fsig


@pytest.mark.parametrize("chunk_batches", [1, 0])
@pytest.mark.parametrize("fp32", [True, False])
def test_static_runs_equal_cls_run(env, fp32, chunk_batches):
    torch, cls = env
    big = Spec(3, (0.6, 1.4), (0.7, 0.95), (0.8, 0.4), 1500, 3_000_000, 6101)
    small = Spec(2, (0.3, 2.0), (0.5, 0.9), (2.0, 0.2), 37, 40_000, 6102)
    cls.cls_set_launch_config(chunk_batches=chunk_batches)
    try:
        for s in (big, small):        # the second call reuses the workspace with a smaller input
            print("static run", "fp32" if fp32 else "fp64", "chunk_batches", chunk_batches, s.d, s.nbins,
                  s.histories, flush=True)
            rec, flux, fsig = _static_run(torch, cls, s, fp32)
            ref, rflux, rfsig = _plain_run(cls, s, fp32)
            for k in COUNTS:
                assert rec[k] == ref[k], (k, rec[k], ref[k])
            for k in ("T", "R", "A", "sigma_T", "sigma_R", "sigma_A"):
                assert rec[k] == ref[k], k
            for k in ("total_flux", "sigma_total_flux"):
                assert abs(rec[k] - ref[k]) <= 1e-11 * abs(ref[k]), k
            np.testing.assert_allclose(flux, rflux, rtol=1e-11, atol=1e-14)
            if chunk_batches:
                assert rec["batches"] == ref["batches"]
                np.testing.assert_allclose(fsig, rfsig, rtol=1e-8, atol=1e-14)
            else:
                # batch-means errors from two batchings of the same histories:
                # in a bin whose error is small against its value (many batches
                # score in it) each has a relative spread of about
                # 1 / sqrt(2 (B - 1)); in sparsely hit bins the estimate is not
                # Gaussian, so those bins are checked through the median only
                b = min(rec["batches"], ref["batches"])
                assert b >= min(256, ref["histories"] // 64)
                assert np.array_equal(fsig > 0, rfsig > 0)
                ok = rfsig > 0
                ratio = fsig[ok] / rfsig[ok]
                dense = ok & (rfsig < 0.01 * np.abs(rflux))
                rd = fsig[dense] / rfsig[dense]
                tol = 8.0 / np.sqrt(2.0 * (b - 1))
                print("batches", rec["batches"], ref["batches"], "flux sigma ratio", ratio.min(), np.median(ratio),
                      ratio.max(), "dense bins", int(dense.sum()), rd.min(), rd.max(), "tolerance", tol, flush=True)
                assert dense.sum() >= 1
                assert np.all(np.abs(rd - 1.0) <= tol)
                assert abs(np.median(ratio) - 1.0) <= 0.05
            assert rec["transmitted"] + rec["reflected"] + rec["absorbed"] == s.histories
    finally:
        cls.cls_set_launch_config(0, 0, 0, 0)


def test_static_run_refuses_what_does_not_fit(env):
    torch, cls = env
    s = Spec(3, (0.6, 1.4), (0.7, 0.95), (0.8, 0.4), 100, 1000, 6103)
    p = gpu_problem(s, fp32=True)
    t = gpu_problem(s, trace=True)
    try:
        buf = torch.zeros(cls.record_bytes(s.nbins) // 8, dtype=torch.int64, device="cuda")
        with pytest.raises(cls.ClsError) as ei:          # record buffer too small
            cls.cls_run_static(p, s.histories, s.seed, None, buf.data_ptr(), cls.record_bytes(s.nbins) - 8)
        assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        with pytest.raises(cls.ClsError) as ei:          # traces need allocated buffers
            cls.cls_run_static(t, s.histories, s.seed, None, buf.data_ptr(), cls.record_bytes(s.nbins))
        assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        with pytest.raises(cls.ClsError) as ei:
            cls.cls_run_static(p, 0, s.seed, None, buf.data_ptr(), cls.record_bytes(s.nbins))
        assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        # a valid mesh whose sums do not fit the static workspace (2048 bins at most)
        fine = gpu_problem(Spec(3, (0.6, 1.4), (0.7, 0.95), (0.8, 0.4), 2049, 1000, 6104), fp32=True)
        try:
            big = torch.zeros(cls.record_bytes(2049) // 8, dtype=torch.int64, device="cuda")
            with pytest.raises(cls.ClsError) as ei:
                cls.cls_run_static(fine, 1000, 6104, None, big.data_ptr(), cls.record_bytes(2049))
            assert ei.value.status == cls.CLS_ERR_INVALID_ARG
        finally:
            cls.cls_destroy_problem(fine)
    finally:
        cls.cls_destroy_problem(p)
        cls.cls_destroy_problem(t)
