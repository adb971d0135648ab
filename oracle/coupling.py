"""CFD coupling of the per-cell chemistry (paper Section 2.1 and the detonation case's source
term) -- TEST INFRASTRUCTURE ONLY.

* ``energy_density``: rho u(C, T) = sum_i C_i U_i(T) with U_i = H_i - R T the molar internal
  energy (equivalently sum_i W_i C_i u_i(T) with mass-specific u_i), or rho h = sum_i C_i H_i(T);
  and its T-derivative rho c_v = sum_i C_i Cv_i (Cv_i = Cp_i - R), or rho c_p = sum_i C_i Cp_i.
* ``T_from_energy``: the temperature that reproduces a given rho u (or rho h), by Newton's method
  with a fixed number of iterations (n = 5 in the paper):
      (d rho u / dT) dT = rho u - rho u(C, T_{k-1}),  T_k = T_{k-1} + dT.
  (The printed update subtracts the quotient; the Newton equation printed just before it, and
  convergence, fix the sign used here.)
* ``openfoam_source``: the linearised production term handed to the species transport equations,
  R_i = W_i (C_i^{n+1} - C_i^n) / dt, in kg/(m^3 s).
"""

from __future__ import annotations

import numpy as np

from .kinetics import CONST_V
from .mechanism import R
from .thermo import nasa7_molar


def energy_density(mech, C, T, energy):
    """(rho u, rho c_v) for energy == CONST_V, (rho h, rho c_p) for CONST_P and CONST_P_REACTOR;
    C [m, ns], T [m]."""
    cp_R, h_RT, _, _, _ = nasa7_molar(mech, np.asarray(T))
    shift = 1.0 if energy == CONST_V else 0.0
    e = (C * (h_RT - shift)).sum(axis=1) * R * T
    de = (C * (cp_R - shift)).sum(axis=1) * R
    return e, de


def T_from_energy(mech, C, e, T0, energy, n_iter=5):
    """Temperatures [m] with energy_density(C, T) = e after n_iter Newton iterations from T0."""
    T = np.array(T0, dtype=float, copy=True)
    for _ in range(n_iter):
        ek, dk = energy_density(mech, C, T, energy)
        T = T + (e - ek) / dk
    return T


def openfoam_source(mech, y_n, y_np1, dt):
    """R_i = W_i (C_i^{n+1} - C_i^n) / dt for every cell ([m, ns]); y = (T, C)."""
    return (np.asarray(y_np1)[:, 1:] - np.asarray(y_n)[:, 1:]) / dt * mech.W[None, :]
