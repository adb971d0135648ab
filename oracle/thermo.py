"""NASA-7 species thermodynamics (paper Section 2.1, Table 1, with n_p = 4).

The paper refits cp to one polynomial of degree n_p and derives h, u, s, g
from it (Table 1).  The NASA-7 two-range form used here is the same family
with n_p = 4 in molar, dimensionless form:

    cp/R  = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
    h/RT  = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
    s0/R  = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7
    g0/RT = h/RT - s0/R

(a6 and a7 play the roles of h_ref and s0_ref.)  The low range applies for
T < T_mid, the high range for T >= T_mid.  Mass-specific values divide the
molar ones by W_i (R_i = R / W_i, Section 2.1).
"""

from __future__ import annotations

import numpy as np

from .mechanism import R


def _coeffs(mech, T):
    """Per-cell, per-species coefficient sets [nc, ns, 7], chosen by the real part of T."""
    Tr = np.real(T)[:, None]
    return np.where((Tr < mech.T_mid[None, :])[:, :, None], mech.nasa_lo[None], mech.nasa_hi[None])


def _poly_molar(a, h0, s0, T):
    """Single-range polynomial cp/R = sum_k a_k T^k (eq. specific_heat_polynomial, molar and
    dimensionless) and what follows from it: h/RT = (h0 + sum_k a_k T^(k+1)/(k+1)) / T (the
    enthalpy identity with h0 the integration constant), s0/R = a_0 ln T + sum_(k>=1) a_k T^k / k
    + s0, and d(cp/R)/dT.  Plain power sums."""
    cp = sum(a[k] * T**k for k in range(len(a)))
    h = (h0 + sum(a[k] * T**(k + 1) / (k + 1) for k in range(len(a)))) / T
    s = a[0] * np.log(T) + sum(a[k] * T**k / k for k in range(1, len(a))) + s0
    dcp = sum(k * a[k] * T**(k - 1) for k in range(1, len(a)))
    return cp, h, s, dcp


def nasa7_molar(mech, T):
    """Return cp/R, h/RT, s0/R, g0/RT, d(cp/R)/dT, each [nc, ns]; T may be complex (complex-step).
    Species with a single-range polynomial cp (``mech.poly``) use that form instead."""
    T = np.asarray(T)
    a = _coeffs(mech, T)
    t = T[:, None]
    a1, a2, a3, a4, a5, a6, a7 = (a[..., k] for k in range(7))
    cp_R = a1 + a2 * t + a3 * t**2 + a4 * t**3 + a5 * t**4
    h_RT = a1 + a2 * t / 2 + a3 * t**2 / 3 + a4 * t**3 / 4 + a5 * t**4 / 5 + a6 / t
    s_R = a1 * np.log(t) + a2 * t + a3 * t**2 / 2 + a4 * t**3 / 3 + a5 * t**4 / 4 + a7
    dcp_R = a2 + 2 * a3 * t + 3 * a4 * t**2 + 4 * a5 * t**3
    for i, (ap, h0, s0) in getattr(mech, "poly", {}).items():
        c, h, s, d = _poly_molar(ap, h0, s0, T)
        cp_R[:, i], h_RT[:, i], s_R[:, i], dcp_R[:, i] = c, h, s, d
    g_RT = h_RT - s_R
    return cp_R, h_RT, s_R, g_RT, dcp_R


T_REF = 298.15


def refit_cp(doc, n_p, T_low=300.0, T_high=3000.0, n_grid=400):
    """Replace every species' NASA-7 data in a mechanism document by a single-range polynomial cp
    of degree n_p (Section 2.1: cp fitted to arbitrary order; Appendix C.1 studies n_p): least
    squares of the NASA-7 cp/R on n_grid Chebyshev points of [T_low, T_high] (numpy.polyfit), then
    the integration constants h0 and s0 set so that h and s equal the NASA-7 values at 298.15 K
    (the enthalpy identity with h_ref at T_ref).  Returns a new document."""
    import copy
    from .mechanism import Mechanism
    out = copy.deepcopy(doc)
    m = Mechanism(doc)
    x = np.cos(np.pi * (np.arange(n_grid) + 0.5) / n_grid)
    Tg = 0.5 * (T_low + T_high) + 0.5 * (T_high - T_low) * x
    cp, _, _, _, _ = nasa7_molar(m, Tg)
    Tr = np.array([T_REF])
    _, h_ref, s_ref, _, _ = nasa7_molar(m, Tr)
    for i, sp in enumerate(out["species"]):
        a = np.polyfit(Tg, cp[:, i], n_p)[::-1]          # a_0 .. a_np
        _, h_no, s_no, _ = _poly_molar(a, 0.0, 0.0, Tr)
        h0 = (h_ref[0, i] - h_no[0]) * T_REF             # h/RT (T_ref) matched
        s0 = s_ref[0, i] - s_no[0]
        sp["thermo"] = {"model": "polynomial-cp", "T-range": [T_low, T_high], "cp-R": [float(v) for v in a],
                        "h0": float(h0), "s0": float(s0)}
    return out


def thermo_mass_specific(mech, T):
    """Mass-specific cp [J/kg/K], h [J/kg], s0 [J/kg/K], g0 [J/kg], each [nc, ns] (Table 1 quantities)."""
    cp_R, h_RT, s_R, g_RT, _ = nasa7_molar(mech, T)
    t = np.asarray(T)[:, None]
    Ri = R / mech.W[None, :]
    return cp_R * Ri, h_RT * Ri * t, s_R * Ri, g_RT * Ri * t
