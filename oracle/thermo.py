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


def nasa7_molar(mech, T):
    """Return cp/R, h/RT, s0/R, g0/RT, d(cp/R)/dT, each [nc, ns]; T may be complex (complex-step)."""
    T = np.asarray(T)
    a = _coeffs(mech, T)
    t = T[:, None]
    a1, a2, a3, a4, a5, a6, a7 = (a[..., k] for k in range(7))
    cp_R = a1 + a2 * t + a3 * t**2 + a4 * t**3 + a5 * t**4
    h_RT = a1 + a2 * t / 2 + a3 * t**2 / 3 + a4 * t**3 / 4 + a5 * t**4 / 5 + a6 / t
    s_R = a1 * np.log(t) + a2 * t + a3 * t**2 / 2 + a4 * t**3 / 3 + a5 * t**4 / 4 + a7
    g_RT = h_RT - s_R
    dcp_R = a2 + 2 * a3 * t + 3 * a4 * t**2 + 4 * a5 * t**3
    return cp_R, h_RT, s_R, g_RT, dcp_R


def thermo_mass_specific(mech, T):
    """Mass-specific cp [J/kg/K], h [J/kg], s0 [J/kg/K], g0 [J/kg], each [nc, ns] (Table 1 quantities)."""
    cp_R, h_RT, s_R, g_RT, _ = nasa7_molar(mech, T)
    t = np.asarray(T)[:, None]
    Ri = R / mech.W[None, :]
    return cp_R * Ri, h_RT * Ri * t, s_R * Ri, g_RT * Ri * t
