"""Writes adjoint_methane_samples.json, the oracle's references for the differentiation workload
on the 53-species mechanism (16,384 cells, seed 2003; backward Euler 500 x 2e-8 s; loss
L = sum_c [T_N + w_c . Y_N], w ~ N(0, 1) seed 3000):

* "adjoint": 3 cells drawn with seed 5003: the oracle's discrete adjoint along its own recorded
  steps, dL/dy0 per cell and dL/dlnA summed over the 3 cells;
* "tangent": the first 64 cells: the oracle's forward (tangent) sensitivities dy_N/d(lnA, y0)
  contracted with dL/dy_N, i.e. dL/dlnA summed over the 64 cells and dL/dy0 per cell.

Calls only oracle/ and the seeded generators.

    python tests/golden/make_adjoint_methane_samples.py
"""

import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N = 16384
DT, STEPS = 1e-5, 500
N_TANGENT = 64


def _load():
    import oracle
    from synth import mechanism_file
    from synth.states import STATE_CONFIGS, loss_weights, sample_states
    om = oracle.load_mechanism(mechanism_file("ch4like_53_325"))
    cfg = STATE_CONFIGS["adjoint_methane"]
    T, p, Y = sample_states(om.ns, N, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    return om, T, p, Y, loss_weights(N, om.ns)


def _adjoint_cell(c):
    import oracle
    from oracle.sensitivity import be_adjoint, final_loss
    om, T, p, Y, w = _load()
    y0 = oracle.state_from_TPY(om, T[c:c + 1], p[c:c + 1], Y[c:c + 1])
    ref = oracle.integrate_be(om, y0, DT, STEPS, record=True)
    _, lamN = final_loss(om, ref["y"], w[c:c + 1])
    lam0, g = be_adjoint(om, lamN, ref["trajectory"])
    return {"cell": int(c), "status": int(ref["status"][0]), "y": ref["y"][0].tolist(), "lamN": lamN[0].tolist(),
            "dLdy0": lam0[0].tolist(), "dLdlnA": g[0].tolist()}


def _tangent_chunk(cells):
    import oracle
    from oracle.sensitivity import be_tangent, final_loss
    om, T, p, Y, w = _load()
    c0, c1 = cells
    y0 = oracle.state_from_TPY(om, T[c0:c1], p[c0:c1], Y[c0:c1])
    ref = oracle.integrate_be(om, y0, DT, STEPS, record=True)
    _, lamN = final_loss(om, ref["y"], w[c0:c1])
    s = be_tangent(om, y0, ref["trajectory"])
    gl = np.einsum("ci,cij->cj", lamN, s)
    return ref["status"].tolist(), gl[:, :om.nr], gl[:, om.nr:]


def main():
    idx = sorted(int(i) for i in np.random.default_rng(5003).choice(N, size=3, replace=False))
    chunks = [(k, k + 8) for k in range(0, N_TANGENT, 8)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        adj = pool.map(_adjoint_cell, idx)
        tan = pool.map(_tangent_chunk, chunks)
    status = sum((t[0] for t in tan), [])
    g_tan = np.concatenate([t[1] for t in tan]).sum(axis=0)
    d0_tan = np.concatenate([t[2] for t in tan])
    out = {"mechanism": "ch4like_53_325", "state_set": "adjoint_methane", "cells_total": N, "dt": DT,
           "n_steps": STEPS, "loss_weight_seed": 3000,
           "adjoint": {"sample_seed": 5003, "cells": adj,
                       "dLdlnA_sum": np.sum([a["dLdlnA"] for a in adj], axis=0).tolist()},
           "tangent": {"cells": list(range(N_TANGENT)), "status": status, "dLdlnA_sum": g_tan.tolist(),
                       "dLdy0": d0_tan.tolist()}}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_methane_samples.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
