"""Single-range polynomial cp for a mechanism (Section 2.1: cp fitted to arbitrary order n_p,
eq. specific_heat_polynomial, h from the enthalpy identity; Appendix C.1 studies n_p = 4, 7, 15).

Host-side preprocessing of a mechanism file: every species' NASA-7 data is replaced by the thermo
model ``polynomial-cp`` -- cp/R = sum_k a_k T^k of degree n_p over one temperature range, fitted by
least squares to the NASA-7 cp/R at Chebyshev points of [T_low, T_high], with the integration
constants h0 and s0 chosen so that h and s keep their NASA-7 values at 298.15 K.  The generated
kernels then evaluate h/RT = sum a_k T^k/(k+1) + h0/T and s/R = a_0 ln T + sum_(k>=1) a_k T^k/k + s0.
"""

from __future__ import annotations

import copy
import json
import math

import numpy as np

T_REF = 298.15


def _nasa7_at(data, t_mid, T):
    """(cp/R, h/RT, s/R) of one NASA-7 species at temperatures T (array)."""
    T = np.asarray(T, dtype=float)
    lo, hi = np.asarray(data[0], dtype=float), np.asarray(data[1], dtype=float)
    c = np.where((T >= t_mid)[:, None], hi[None, :], lo[None, :])
    cp = c[:, 0] + T * (c[:, 1] + T * (c[:, 2] + T * (c[:, 3] + T * c[:, 4])))
    h = c[:, 0] + T * (c[:, 1] / 2 + T * (c[:, 2] / 3 + T * (c[:, 3] / 4 + T * c[:, 4] / 5))) + c[:, 5] / T
    s = c[:, 0] * np.log(T) + T * (c[:, 1] + T * (c[:, 2] / 2 + T * (c[:, 3] / 3 + T * c[:, 4] / 4))) + c[:, 6]
    return cp, h, s


def refit_document(doc: dict, n_p: int, T_low: float = 300.0, T_high: float = 3000.0, n_grid: int = 400) -> dict:
    """A copy of the mechanism document with every NASA-7 species refitted to degree n_p."""
    if n_p < 1 or not (T_high > T_low > 0.0):
        raise ValueError("n_p >= 1 and 0 < T_low < T_high required")
    out = copy.deepcopy(doc)
    j = np.arange(n_grid)
    Tg = 0.5 * (T_low + T_high) + 0.5 * (T_high - T_low) * np.cos(math.pi * (j + 0.5) / n_grid)
    for sp in out["species"]:
        th = sp["thermo"]
        if th["model"] != "NASA7":
            continue
        t_mid = float(th["temperature-ranges"][1])
        cp, _, _ = _nasa7_at(th["data"], t_mid, Tg)
        a = np.polyfit(Tg, cp, n_p)[::-1]
        _, h_ref, s_ref = _nasa7_at(th["data"], t_mid, np.array([T_REF]))
        h_poly = sum(a[k] * T_REF ** k / (k + 1) for k in range(n_p + 1))          # h/RT without h0
        s_poly = a[0] * math.log(T_REF) + sum(a[k] * T_REF ** k / k for k in range(1, n_p + 1))
        sp["thermo"] = {"model": "polynomial-cp", "T-range": [T_low, T_high], "cp-R": [float(v) for v in a],
                        "h0": float((h_ref[0] - h_poly) * T_REF), "s0": float(s_ref[0] - s_poly)}
    return out


def refit_file(src: str, dst: str, n_p: int, **kw) -> str:
    """Write the refit of mechanism file ``src`` to ``dst`` (JSON) and return ``dst``."""
    with open(src) as f:
        doc = json.load(f)
    with open(dst, "w") as f:
        json.dump(refit_document(doc, n_p, **kw), f, indent=1)
    return dst
