"""Algorithmic operation counts of the generated kernels, for roofline reporting.

Counts follow the arithmetic the code generator emits for a mechanism, construct by construct:
+, -, *, / count 1 flop each, a fused multiply-add counts 2; exp, log and sqrt are counted
separately as transcendental operations ("T-ops") and contribute no flops (a T-op is a
multi-instruction routine of the device math library, so its internal instructions are not
algorithmic work of the method).  Selects, comparisons, loads and sign flips count 0.

The result is the work per unit of the method -- one source-term evaluation, one Jacobian, one
Rosenbrock attempt, one Newton iteration -- that the benchmark multiplies by the units a
launch processed.
"""

from __future__ import annotations

import json
from dataclasses import dataclass


@dataclass
class Count:
    flops: float = 0.0
    tops: float = 0.0

    def __add__(self, o):
        return Count(self.flops + o.flops, self.tops + o.tops)

    def __mul__(self, k):
        return Count(self.flops * k, self.tops * k)


def _net(rx):
    nu = {}
    for s, c in rx["reactants"].items():
        nu[s] = nu.get(s, 0) - int(c)
    for s, c in rx["products"].items():
        nu[s] = nu.get(s, 0) + int(c)
    return {s: v for s, v in nu.items() if v != 0}


def _rate_count(rx, jac: bool) -> Count:
    c = Count()
    kind = rx["type"]
    k = rx["rate-constant"] if "rate-constant" in rx else rx["high-P-rate-constant"]
    c.flops += (2 if k["b"] != 0 else 0) + (2 if k["Ea"] != 0 else 0)      # lnk
    pd = kind != "elementary"
    if pd:
        eff = [v for v in rx.get("efficiencies", {}).values() if v != rx.get("default-efficiency", 1.0)]
        c.flops += 2 * len(eff) + (1 if rx.get("default-efficiency", 1.0) not in (0.0, 1.0) else 0)
    if kind == "elementary":
        c.tops += 1
    elif kind == "three-body":
        c.tops += 1
        c.flops += 1
    else:
        c.flops += 4 + 1 + 1 + 3           # ln ratio, Pr, 1 + Pr, kinf * (Pr/(1+Pr)) * F
        c.tops += 2
        if "Troe" in rx:
            has_t2 = "T2" in rx["Troe"]
            c.tops += 2 + (1 if has_t2 else 0) + 2 + 1          # e3 e1 [e2], log Fc, log Pr, exp F
            c.flops += 2 + (1 if has_t2 else 0) + 3 + (1 if has_t2 else 0) + 2 + 2 + 2 + 1 + 2 + 1 + 3 + 2
            if jac:
                c.flops += 4 + 2 + 2 + 6 + 3 + 5 + (4 if has_t2 else 0)
        if jac:
            c.flops += 3 + 3 + 6 + 3
    nf = sum(int(v) for v in rx["reactants"].values())
    nrv = sum(int(v) for v in rx["products"].values())
    nu = _net(rx)
    c.flops += nf                                                   # Rf
    rev = rx.get("reversible", True)
    if rev:
        dnu = sum(nu.values())
        c.flops += max(0, len(nu) - 1) + sum(1 for v in nu.values() if abs(v) != 1)
        c.flops += 3 if dnu != 0 else 0
        c.tops += 1
        c.flops += 1 + nrv                                          # kr, Rr
    c.flops += 1                                                    # q
    if not jac:
        return c
    c.flops += sum(1 if abs(v) == 1 else 2 for v in nu.values())   # omega scatter
    c.flops += 3 if kind != "falloff" else 0                        # dlnkf/dT
    if rev:
        c.flops += max(0, len(nu) - 1) + sum(1 for v in nu.values() if abs(v) != 1) + 2   # dlnKc/dT
        c.flops += 3                                                # dq/dT
    else:
        c.flops += 1
    cols = set()
    for side in (rx["reactants"], rx["products"] if rev else {}):
        for s, v in side.items():
            c.flops += max(0, sum(int(x) for x in side.values()) - 1) + (1 if int(v) > 1 else 0)
            if s in cols:
                c.flops += 1
            cols.add(s)
    if pd:
        c.flops += 1                                                # qM
        for s in rx.get("efficiencies", {}):
            c.flops += 2 if s not in cols else 3
            cols.add(s)
        c.flops += 2 * len(nu)                                      # dense third-body row accumulators
    c.flops += sum((1 if abs(v) == 1 else 2) * (1 + len(cols)) for v in nu.values())   # J scatter
    return c


class MechanismCounts:
    def __init__(self, path: str):
        with open(path) as f:
            self.doc = json.load(f)
        self.ns = len(self.doc["species"])
        self.n = self.ns + 1
        self.rx = self.doc["reactions"]
        self.any_pd = any(r["type"] != "elementary" for r in self.rx)
        active = set()
        for r in self.rx:
            active |= set(_net(r))
        # integrators solve only T and the species that change (the others have zero increments)
        self.ns_active = len(active)
        self.na = self.ns_active + 1

    def source(self) -> Count:
        ns = self.ns
        c = Count(flops=1, tops=1)                                  # invT, lnT
        c.flops += 37 * ns                                          # NASA-7 cp, h, s, g in Horner form
        if self.any_pd:
            c.flops += ns - 1
        for r in self.rx:
            c = c + _rate_count(r, False)
            c.flops += sum(1 if abs(v) == 1 else 2 for v in _net(r).values())
        c.flops += 6 * ns + 2                                       # omega_T
        return c

    def jacobian(self, reduced: bool = False) -> Count:
        """Full Jacobian (API kernel), or the active-component one the integrators factor."""
        ns = self.ns
        cols = self.ns_active if reduced else ns
        c = Count(flops=1, tops=1)
        c.flops += 46 * ns
        if self.any_pd:
            c.flops += ns - 1 + self.ns_active * cols               # M_c, dense third-body part
        for r in self.rx:
            c = c + _rate_count(r, True)
        c.flops += 6 * ns + 2
        c.flops += 3 + 4 * ns + 2 * self.ns_active + 5 + cols * (2 * self.ns_active + 4)   # temperature row
        return c

    def lu(self, n=None) -> Count:
        n = self.na if n is None else n
        return Count(flops=sum(1 + (n - k - 1) + 2 * (n - k - 1) ** 2 for k in range(n)))

    def solve(self, n=None) -> Count:
        n = self.na if n is None else n
        return Count(flops=2 * n * (n - 1) + n)

    def ros2_attempt(self) -> Count:
        n, ns = self.na, self.ns
        c = self.jacobian(reduced=True) + self.lu() + self.solve() * 2 + self.source()
        c.flops += 2 + n                                            # 1/(gamma h), G = d I - J
        c.flops += 2 * n + 2 * n + 1                                # y*, rhs of stage 2
        c.flops += 4 * n + 2 * n                                    # y_new, error vector
        c.flops += 4 + 11 * ns + 2                                  # weighted RMS error
        c.tops += 2                                                 # sqrt(err), sqrt in the factor
        c.flops += 6                                                # controller
        return c

    def sdirk_iteration(self) -> Count:
        """One Newton iteration of an SDIRK stage (Appendix A.1, A.2) on the active system (the
        initial guess S(y_n) of each step is one source() evaluation, counted by the caller)."""
        n, ns = self.na, self.ns
        c = self.jacobian(reduced=True) + self.lu() + self.solve()
        c.flops += 2 * n + 1 + n                                    # stage state b + gamma h Gamma, gamma h
        c.flops += n + n * n + n                                    # residual, G = I - gamma h J
        c.flops += 2 * n + n + 5 * ns + 3                           # update, scaled norm
        return c

    def sdirk_step_combination(self, stages: int) -> Count:
        """Per completed SDIRK step: the stage bases b_p = y_n + sum_{j<p} (h a_pj) Gamma_j and
        y_{n+1} = y_n + sum_p (h b_p) Gamma_p on the active components (one multiply and one add
        per term; the products h a_pj and h b_p once each)."""
        n = self.na
        terms = stages * (stages - 1) // 2 + stages
        return Count(flops=2 * n * terms + terms + 1)

    def be_iteration(self) -> Count:
        n, ns = self.na, self.ns
        c = self.jacobian(reduced=True) + self.lu() + self.solve()
        c.flops += 1 + 1 + n + 3 * n                                # h, 1/h, G, residual
        c.flops += n + 3 + 6 * ns                                   # update, scaled norm
        return c


if __name__ == "__main__":
    import sys
    m = MechanismCounts(sys.argv[1])
    for name in ("source", "jacobian", "lu", "ros2_attempt", "be_iteration", "sdirk_iteration"):
        v = getattr(m, name)()
        print(f"{name:14s} flops {v.flops:10.0f}  T-ops {v.tops:6.0f}")
