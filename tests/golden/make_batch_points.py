"""Writes tests/golden/batch_points.json: FP64 oracle linewidths at sampled
first-mode points of the three costliest crystals of the 32-crystal batch
(cells of 54, 49 and 36 atoms on 9^3, 9^3 and 10^3 grids), T = 300 K,
Gaussian delta of 0.1 THz.  Calls only the oracle and the seeded generator.

Run from the repository root:  python tests/golden/make_batch_points.py
(about a quarter of an hour on 8 host cores)."""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import batch_crystals  # noqa: E402
from oracle import phonons as P, anharmonic as A  # noqa: E402

T, SIGMA = [300.0], 0.1
CRYSTALS = (1, 17, 8)       # indices in the batch: the three largest projection costs
POINTS = (1, 100)           # first-mode points sampled in each


def main():
    crystals = batch_crystals()
    out = {"T": T, "sigma_thz": SIGMA, "generator": "gen.batch_crystals() (seeded)", "crystals": []}
    for ci in CRYSTALS:
        c = crystals[ci]
        t0 = time.perf_counter()
        ph = P.phonons(c, velocities=False)
        g = A.linewidths(c, ph, T, SIGMA, k_subset=list(POINTS))
        print(f"{c.name}: {time.perf_counter() - t0:.0f} s", flush=True)
        out["crystals"].append({"index": ci, "name": c.name, "points": list(POINTS),
                                "gamma": g[0].tolist(), "mask": ph.mask[list(POINTS)].tolist()})
    path = os.path.join(ROOT, "tests", "golden", "batch_points.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
