"""Pins of the oracle's random numbers.

* The Philox4x32-10 bijection (Salmon et al., SC'11) is checked bitwise against
  rocRAND's independent implementation, run on the same counters and keys.
* The uniform mapping U = (k + 1/2) 2^-23 is checked for range, exactness in FP32,
  uniformity (chi-square) and independence of the five uniforms of a block and of
  adjacent blocks (correlation), so that a wrong shift, mask or offset fails.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("ref") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(99)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0),
             (0, 0, 0, 0, 0, 1)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, 6)) for _ in range(2000)]
    inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(map(int, l.split())) for l in out.strip().split("\n")]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        assert oracle.philox4x32_10(c[:4], c[4:]) == r, c


def _uniforms(n_hist, steps, seed=12345):
    u = np.empty((n_hist * steps, 5))
    i = 0
    for h in range(n_hist):
        for j in range(steps):
            u[i] = oracle.step_uniforms(seed, h, j)
            i += 1
    return u


def test_uniform_range_and_fp32_exactness():
    u = _uniforms(200, 20)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    # (k + 1/2) 2^-23 grid
    k = u * 2.0**23 - 0.5
    assert np.all(k == np.round(k))
    assert u.min() >= 2.0**-24 and u.max() <= 1.0 - 2.0**-24


def test_uniform_distribution_and_independence():
    u = _uniforms(2000, 25)          # 50,000 blocks, 250,000 uniforms
    n = u.shape[0]
    nb = 64
    for i in range(5):
        cnt = np.histogram(u[:, i], bins=nb, range=(0, 1))[0]
        stat = ((cnt - n / nb) ** 2 / (n / nb)).sum()
        assert chi2.sf(stat, nb - 1) > 1e-4, (i, stat)
        assert abs(u[:, i].mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    # the five uniforms of a block are uncorrelated, and so are consecutive blocks
    c = np.corrcoef(u.T)
    off = c[~np.eye(5, dtype=bool)]
    assert np.all(np.abs(off) < 5 / np.sqrt(n)), c
    lag = np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]
    assert abs(lag) < 5 / np.sqrt(n)
    # uniform 4 is assembled from low bits of words 0, 1, 2: its top bits must be
    # independent of the top bits of uniforms 0..2 (2-D chi-square on 8x8 cells)
    for j in range(3):
        h2 = np.histogram2d(u[:, 4], u[:, j], bins=8, range=[[0, 1], [0, 1]])[0]
        stat = ((h2 - n / 64) ** 2 / (n / 64)).sum()
        assert chi2.sf(stat, 63) > 1e-4, (j, stat)


def test_streams_differ_by_history_step_lane_and_seed():
    a = oracle.step_uniforms(1, 0, 0)
    assert not np.array_equal(a, oracle.step_uniforms(1, 1, 0))
    assert not np.array_equal(a, oracle.step_uniforms(1, 0, 1))
    assert not np.array_equal(a, oracle.step_uniforms(1, 0, 0, 1))
    assert not np.array_equal(a, oracle.step_uniforms(2, 0, 0))
    assert not np.array_equal(oracle.step_uniforms(1, 2**32, 0), oracle.step_uniforms(1, 0, 0))
