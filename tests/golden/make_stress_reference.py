"""Write tests/golden/stress3d_oracle_1e6.json: the FP64 oracle on every
stress3d parameter set (d=3 cube, c in [0.99, 0.999]) with 10^6 histories each.

Calls only the oracle; the GPU path never contributes to the stored values.
Run from the repository root:  python tests/golden/make_stress_reference.py
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from helpers import run_oracle                      # noqa: E402
from paper_1708_00765_amd.inputs import workload    # noqa: E402

HISTORIES = 1_000_000
ORACLE_SEED_SALT = 0x0123456789ABCDEF
BIN_EVERY = 4          # per-bin flux is stored for every 4th set (keeps the file small)


def _r(v: float) -> float:
    return float(f"{v:.10g}")


def main() -> None:
    out = []
    t0 = time.time()
    for j, s in enumerate(workload("stress3d", histories=HISTORIES)):
        seed = s.seed ^ ORACLE_SEED_SALT
        r = run_oracle(s, seed=seed)
        rec = {"name": s.name, "sigma": s.sigma, "c": s.c, "lam": s.lam, "nbins": s.nbins,
               "histories": r.histories, "seed": seed, "T": r.T, "sigma_T": r.sigma_T, "R": r.R,
               "sigma_R": r.sigma_R, "A": r.A, "sigma_A": r.sigma_A, "total_flux": r.total_flux,
               "sigma_total_flux": r.total_flux_sigma, "flights": r.flights}
        if j % BIN_EVERY == 0:
            rec["flux"] = [_r(v) for v in r.flux]
            rec["flux_sigma"] = [_r(v) for v in r.flux_sigma]
        out.append(rec)
        print(f"{s.name}: {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(ROOT, "tests", "golden", "stress3d_oracle_1e6.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_stress_reference.py", "histories_per_set": HISTORIES,
                   "sets": out}, f)


if __name__ == "__main__":
    main()
