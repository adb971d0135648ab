"""Mechanism file reader for the oracle (its own parser; the HIP library has another).

The file is Cantera-like JSON: species with NASA-7 data, reactions of type
``elementary``, ``three-body``, ``falloff`` (Troe, SRI or Lindemann) or
``pressure-dependent-Arrhenius`` (P-log: Arrhenius sets at given pressures), rate
constants {A, b, Ea} in SI-kmol units with Ea in J/kmol (the paper's worked
example H + O2 <=> O + OH uses A = 1.0399e11, Ea = 6.405704e7, Section 4.3).
"""

from __future__ import annotations

import json
import math
from dataclasses import dataclass

import numpy as np

R = 8314.462618  # J/(kmol K)


@dataclass
class Reaction:
    kind: str                 # "elementary" | "three-body" | "falloff"
    reactants: dict           # species index -> integer coefficient (nu^f)
    products: dict            # species index -> integer coefficient (nu^r)
    reversible: bool
    lnA: float                # ln of the (high-pressure) prefactor
    b: float
    theta: float              # Ea / R  [K]
    lnA0: float = 0.0         # falloff low-pressure limit
    b0: float = 0.0
    theta0: float = 0.0
    troe: tuple | None = None  # (alpha, T3, T1, T2 or None)
    sri: tuple | None = None   # (a, b, c, d, e) of the SRI broadening
    plog: list | None = None   # P-log: [(ln p_i, ln A_i, b_i, theta_i)] sorted by pressure
    eff: np.ndarray | None = None  # third-body efficiencies alpha_ij (dense, default 1)


class Mechanism:
    def __init__(self, doc: dict):
        self.doc = doc
        sp = doc["species"]
        self.names = [s["name"] for s in sp]
        self.ns = len(sp)
        self.n = self.ns + 1
        idx = {nm: i for i, nm in enumerate(self.names)}
        self.W = np.array([float(s["molecular-weight"]) for s in sp])
        self.inert = np.array([bool(s.get("inert", False)) for s in sp])
        self.elements = [e["symbol"] for e in doc["elements"]]
        self.E = np.array([[s["composition"].get(e, 0) for s in sp] for e in self.elements], dtype=float)
        self.p_ref = float(doc.get("reference-pressure", 101325.0))
        lo, hi, tmid = [], [], []
        self.poly = {}        # species index -> (cp/R coefficients a_0..a_np, h0, s0)
        for i, s in enumerate(sp):
            th = s["thermo"]
            if th["model"] == "polynomial-cp":
                self.poly[i] = (np.array([float(v) for v in th["cp-R"]]), float(th["h0"]), float(th["s0"]))
                tmid.append(1000.0)
                lo.append([0.0] * 7)
                hi.append([0.0] * 7)
                continue
            assert th["model"] == "NASA7"
            tmid.append(float(th["temperature-ranges"][1]))
            lo.append([float(v) for v in th["data"][0]])
            hi.append([float(v) for v in th["data"][1]])
        self.nasa_lo = np.array(lo)
        self.nasa_hi = np.array(hi)
        self.T_mid = np.array(tmid)
        self.reactions = []
        for r in doc["reactions"]:
            reac = {idx[k]: int(v) for k, v in r["reactants"].items()}
            prod = {idx[k]: int(v) for k, v in r["products"].items()}
            kind = r["type"]
            rx = Reaction(kind, reac, prod, bool(r.get("reversible", True)), 0.0, 0.0, 0.0)
            if kind == "falloff":
                hi_k, lo_k = r["high-P-rate-constant"], r["low-P-rate-constant"]
                rx.lnA, rx.b, rx.theta = math.log(hi_k["A"]), float(hi_k["b"]), float(hi_k["Ea"]) / R
                rx.lnA0, rx.b0, rx.theta0 = math.log(lo_k["A"]), float(lo_k["b"]), float(lo_k["Ea"]) / R
                if "Troe" in r:
                    t = r["Troe"]
                    rx.troe = (float(t["A"]), float(t["T3"]), float(t["T1"]),
                               float(t["T2"]) if "T2" in t else None)
                elif "SRI" in r:
                    t = r["SRI"]
                    rx.sri = (float(t["A"]), float(t["B"]), float(t["C"]), float(t.get("D", 1.0)),
                              float(t.get("E", 0.0)))
            elif kind == "pressure-dependent-Arrhenius":
                sets = sorted((math.log(float(k["P"])), math.log(k["A"]), float(k["b"]), float(k["Ea"]) / R)
                              for k in r["rate-constants"])
                rx.kind = kind = "plog"
                rx.plog = sets
                rx.lnA, rx.b, rx.theta = sets[0][1], sets[0][2], sets[0][3]
            else:
                k = r["rate-constant"]
                rx.lnA, rx.b, rx.theta = math.log(k["A"]), float(k["b"]), float(k["Ea"]) / R
            if kind == "plog":
                rx.eff = np.ones(self.ns)             # p = R T sum_i C_i: every species counts once
            if kind in ("three-body", "falloff"):
                eff = np.full(self.ns, float(r.get("default-efficiency", 1.0)))
                for k, v in r.get("efficiencies", {}).items():
                    eff[idx[k]] = float(v)
                rx.eff = eff
            self.reactions.append(rx)
        self.nr = len(self.reactions)
        self.nu_f = np.zeros((self.ns, self.nr))
        self.nu_r = np.zeros((self.ns, self.nr))
        for j, rx in enumerate(self.reactions):
            for i, v in rx.reactants.items():
                self.nu_f[i, j] = v
            for i, v in rx.products.items():
                self.nu_r[i, j] = v
        self.nu = self.nu_r - self.nu_f          # nu_ij = nu^r_ij - nu^f_ij (Section 2.2)
        self.lnA_default = np.array([rx.lnA for rx in self.reactions])


def load_mechanism(path: str) -> Mechanism:
    with open(path) as f:
        return Mechanism(json.load(f))
