"""Writes ros2_methane_samples.json: the oracle's adaptive Rosenbrock integration (rtol 1e-6,
atol 1e-10, one split step of 1e-5 s) of 8 cells drawn (seed 5002) from the 4,096-cell set of the
53-species workload's distribution and seed (sample_config("ros2_methane", 53, 4096): T0 ~
U[800, 2600] K, Dirichlet(0.5), seed 2002), one process per cell.  Calls only oracle/ and the
seeded state generators; takes several minutes per cell.

    python tests/golden/make_ros2_methane_samples.py
"""

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SUBSET = 4096
N_SAMPLES = 8
SEED = 5002
DT = 1e-5


def sample_indices():
    return sorted(int(i) for i in np.random.default_rng(SEED).choice(SUBSET, N_SAMPLES, replace=False))


def _one(c):
    import oracle
    from synth import mechanism_file
    from synth.states import sample_config
    om = oracle.load_mechanism(mechanism_file("ch4like_53_325"))
    T, p, Y = sample_config("ros2_methane", om.ns, SUBSET)
    y0 = oracle.state_from_TPY(om, T[c:c + 1], p[c:c + 1], Y[c:c + 1])
    r = oracle.integrate_ros2(om, y0, DT)
    return {"cell": c, "y": [float(v) for v in r["y"][0]], "status": int(r["status"][0]),
            "accepted": int(r["accepted"][0]), "rejected": int(r["rejected"][0])}


def main():
    idx = sample_indices()
    with Pool(min(len(idx), os.cpu_count() or 1)) as pool:
        rows = pool.map(_one, idx)
    out = {"mechanism": "ch4like_53_325", "state_set": "ros2_methane", "subset": SUBSET, "sample_seed": SEED,
           "dt": DT, "rtol": 1e-6, "atol": 1e-10, "cells": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ros2_methane_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
