"""Pins of the oracle's CFD coupling (temperature from the energy density, OpenFOAM-style source).

* rho c_v and rho c_p equal complex-step T-derivatives of rho u(C, T) and rho h(C, T), and
  rho h - rho u = R T sum C (the ideal-gas relation h = u + R T per mole);
* round trip: from rho u(C, T*) (and rho h) Newton recovers T* to rounding in 5 iterations from
  guesses 300 K away, with the quadratic error decay of Newton's method;
* a mixture whose heat capacities are constant (NASA-7 with only a1, a6) has rho u linear in T:
  one iteration lands on T* exactly (to rounding);
* the source term: on the linear isomerisation with the backward-Euler closed form
  C^{n+1} = (I - hK)^-1 C^n it equals W ((I - hK)^-1 - I) C^n / h; mass is conserved
  (sum_i R_i = 0) and R -> W omega as dt -> 0.
"""

import copy

import numpy as np
import pytest

import oracle
from oracle.coupling import T_from_energy, energy_density, openfoam_source
from oracle.kinetics import CONST_P, CONST_V
from oracle.mechanism import R
from synth.states import sample_config

from test_oracle_integrators import _isomer_mech, _linear_K


def _states(m, n=12):
    T, p, Y = sample_config("ros2_1m", m.ns, n)
    return oracle.state_from_TPY(m, T, p, Y)


@pytest.mark.parametrize("energy", [CONST_V, CONST_P])
def test_heat_capacity_is_the_derivative(mech_small, energy):
    y = _states(mech_small)
    C, T = y[:, 1:], y[:, 0]
    h = 1e-30
    e_c, _ = energy_density(mech_small, C.astype(complex), T + 1j * h, energy)
    _, de = energy_density(mech_small, C, T, energy)
    np.testing.assert_allclose(de, e_c.imag / h, rtol=1e-13)


def test_enthalpy_minus_internal_energy(mech_small):
    y = _states(mech_small)
    C, T = y[:, 1:], y[:, 0]
    u, _ = energy_density(mech_small, C, T, CONST_V)
    hh, _ = energy_density(mech_small, C, T, CONST_P)
    np.testing.assert_allclose(hh - u, R * T * C.sum(axis=1), rtol=1e-10)


@pytest.mark.parametrize("energy", [CONST_V, CONST_P])
@pytest.mark.parametrize("offset", [-300.0, 300.0])
def test_round_trip_and_quadratic_convergence(mech_small, energy, offset):
    y = _states(mech_small)
    C, Tstar = y[:, 1:], y[:, 0]
    e, _ = energy_density(mech_small, C, Tstar, energy)
    T5 = T_from_energy(mech_small, C, e, Tstar + offset, energy)
    np.testing.assert_allclose(T5, Tstar, rtol=1e-13)
    errs = [np.abs(T_from_energy(mech_small, C, e, Tstar + offset, energy, k) - Tstar).max() for k in range(4)]
    assert errs[1] < errs[0] and errs[2] < 0.1 * errs[1]
    if errs[2] > 1e-6:                     # above rounding: the quadratic law e_{k+1} ~ c e_k^2
        assert errs[3] <= 10 * errs[2] ** 2 / errs[1] ** 2 * errs[2]


def test_constant_heat_capacity_one_iteration():
    m = copy.deepcopy(_isomer_mech())
    m.nasa_lo[:, 1:5] = 0.0                       # cp/R = a1: constant
    m.nasa_hi[:, 1:5] = 0.0
    y = np.array([[1400.0, 0.006, 0.001, 0.002]])
    C, Tstar = y[:, 1:], y[:, 0]
    e, _ = energy_density(m, C, Tstar, CONST_V)
    T1 = T_from_energy(m, C, e, np.array([900.0]), CONST_V, n_iter=1)
    np.testing.assert_allclose(T1, Tstar, rtol=1e-14)


def test_openfoam_source_closed_form_and_mass():
    m = _isomer_mech()
    T = 1400.0
    y0 = np.array([[T, 0.006, 0.001, 0.002]])
    K = _linear_K(m, T)
    h = 1e-7
    r = oracle.integrate_be(m, y0, h, 1)
    Rsrc = openfoam_source(m, y0, r["y"], h)
    ref = m.W * ((np.linalg.inv(np.eye(3) - h * K) - np.eye(3)) @ y0[0, 1:]) / h
    np.testing.assert_allclose(Rsrc[0], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    assert abs(Rsrc.sum()) <= 1e-12 * np.abs(Rsrc).max()
    # dt -> 0: R -> W omega
    for dt in (1e-12,):
        r = oracle.integrate_be(m, y0, dt, 1)
        w = oracle.source_terms(m, y0)[0, 1:]
        np.testing.assert_allclose(openfoam_source(m, y0, r["y"], dt)[0], m.W * w, rtol=1e-4)
