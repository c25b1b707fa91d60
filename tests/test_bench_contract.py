"""bench.py's output contract: one JSON line with the metric, the roofline of the
tracking kernel and the oracle baseline; more than one GPU is refused."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout


@pytest.mark.gpu
def test_bench_line_on_a_small_run():
    """A reduced run of the stress3d sets (1e6 histories per set, FP64 leg, 1 s of
    oracle) prints the
    JSON line with every field the benchmark reports; the measured traffic is
    only reported for the full workload."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0",
           "--histories", "1000000", "--fp64-steps", "1", "--cpu-seconds", "1", "--serve-seconds", "0",
           "--saturate-seconds", "0", "--ext2d-steps", "0", "--quenched-histories", "0", "--cube3d-steps", "0"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    print(r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    j = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in j, k
    assert j["n_gpus"] == 1 and j["steps"] == 1 and j["warmup"] == 0
    assert j["value"] > 0 and j["ms_per_step"] > 0 and j["higher_is_better"] is True
    assert j["unit"] == "histories/s" and j["data"] == "synthetic" and j["vs_baseline"] is None
    assert "workload" in j["config"]
    roof = j["roofline"]
    assert roof["bound"] == "alu" and roof["unit"] == "Tslot/s"
    assert 0 < roof["achieved"] <= roof["peak"] and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9
    assert roof["traffic"] is None          # recorded for the full workload only
    cpu = j["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["unit"] == "histories/s"
    assert isinstance(cpu["sample"], str) and cpu["sample"]
    assert j["fp64_plain"]["value"] > 0
    lc = j["launch_config"]            # the autotuned configuration, the default one timed beside it
    assert lc["default_config_value"] > 0 and set(lc["autotuned_config"]) == {
        "waves_per_block", "blocks_per_cu", "max_chunk", "refill_min", "slots", "chunk_batches"}
    acc = j["fp32_vs_fp64_same_streams"]
    assert acc["bins_compared"] == 32 * 1000 and set(acc["violations"]) == {"scalars", "profiles", "bins"}
    orc = j["fp32_vs_oracle"]
    assert orc["bins"] > 0 and orc["oracle_histories_per_set"] > 0
