"""Writes tests/golden/sige648.json: FP64 oracle linewidths of every mode of the
disordered Si(0.5)Ge(0.5) cell of 3^3 conventional cells (216 atoms, 648
modes, Gamma point), T = 300 K, Gaussian delta of 0.1 THz, with the oracle's
frequencies.  Calls only the oracle and the seeded generator.

Run from the repository root:  python tests/golden/make_sige648.py
(a few minutes on 8 host cores)."""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import sige_supercell  # noqa: E402
from oracle import phonons as P, anharmonic as A  # noqa: E402

T, SIGMA = [300.0], 0.1


def main():
    c = sige_supercell(reps=3)
    t0 = time.perf_counter()
    ph = P.phonons(c, velocities=False)
    g = A.linewidths_gamma_sparse(c, ph, T, SIGMA)
    print(f"{c.name}: {c.n_modes} modes, {time.perf_counter() - t0:.0f} s", flush=True)
    out = {"crystal": "sige_supercell(reps=3)", "T": T, "sigma_thz": SIGMA,
           "omega": ph.omega[0].tolist(), "gamma": g.tolist()}
    path = os.path.join(ROOT, "tests", "golden", "sige648.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
