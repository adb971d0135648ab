"""Pins of the oracle's SDIRK-2 (Appendix A.1) against independent facts.

* linear isomerisation A <=> B (T constant, dC/dt = K C): one step is the stability function
  R(z) = (1 + (1 - 2 gamma) z) / (1 - gamma z)^2 applied to hK (derived from the two stage
  equations for y' = lambda y), so N steps equal (R(hK))^N y0 to rounding, and the scheme
  converges to expm(K t) at order 2;
* R is L-stable with gamma = 1 - sqrt(2)/2: |R(z)| <= 1 on the negative axis and R(z) -> 0;
* order 2 on a synthetic mechanism against a fine Rosenbrock reference;
* linear invariants (element totals, mass, inert species) are kept;
* a step whose Newton iteration cannot converge sets CELL_NEWTON_FAIL and keeps the state.
"""

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle.integrate import SDIRK2_GAMMA, IntegratorOptions
from synth.states import sample_config

from test_oracle_integrators import _isomer_mech, _linear_K, _onto_manifold

G = SDIRK2_GAMMA


def _R_matrix(hK):
    I = np.eye(hK.shape[0])
    A = np.linalg.inv(I - G * hK)
    return A @ A @ (I + (1.0 - 2.0 * G) * hK)


def test_linear_isomerisation_closed_form_and_order():
    m = _isomer_mech()
    T = 1400.0
    y0 = np.array([[T, 0.006, 0.001, 0.002]])
    K = _linear_K(m, T)
    tend = 0.5 / abs(K[0, 0])
    exact = expm(K * tend) @ y0[0, 1:]
    errs = []
    for N in (8, 16, 32, 64):
        h = tend / N
        r = oracle.integrate_sdirk2(m, y0, tend, N)
        assert r["status"][0] == 0
        np.testing.assert_allclose(r["y"][0, 0], T, rtol=0, atol=1e-9)
        ref = np.linalg.matrix_power(_R_matrix(h * K), N) @ y0[0, 1:]
        np.testing.assert_allclose(r["y"][0, 1:], ref, rtol=1e-12, atol=1e-18)
        errs.append(np.abs(r["y"][0, 1:] - exact).max())
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(o - 2.0) < 0.2) and abs(o[-1] - 2.0) < 0.1, o


def test_stability_function_is_l_stable():
    z = -np.logspace(-3, 8, 200)
    Rz = (1 + (1 - 2 * G) * z) / (1 - G * z) ** 2
    assert np.all(np.abs(Rz) <= 1.0)
    assert abs(Rz[-1]) < 1e-7


def test_convergence_order_on_mechanism(mech_small):
    m = mech_small
    y0 = _onto_manifold(m)
    t = 2e-9
    ref = oracle.integrate_ros2(m, y0, t, fixed_steps=512)["y"]
    e = []
    # errors from 1e-13 down to 2e-15 (finer steps reach the reference's own error)
    for N in (8, 16, 32, 64):
        r = oracle.integrate_sdirk2(m, y0, t, N)
        assert np.all(r["status"] == 0)
        e.append(np.abs(r["y"][:, 1:] - ref[:, 1:]).max())
    o = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.median(o) == pytest.approx(2.0, abs=0.3), o


def test_invariants(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 6)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    r = oracle.integrate_sdirk2(m, y0, 2e-6, 20)
    assert np.all(r["status"] == 0)
    y = r["y"]
    np.testing.assert_allclose(y[:, 1:] @ m.E.T, y0[:, 1:] @ m.E.T, rtol=1e-11)
    np.testing.assert_allclose(y[:, 1:] @ m.W, y0[:, 1:] @ m.W, rtol=1e-12)
    inert = 1 + np.nonzero(m.inert)[0]
    np.testing.assert_allclose(y[:, inert], y0[:, inert], rtol=1e-13)


def test_newton_failure_status(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 3)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    r = oracle.integrate_sdirk2(m, y0, 1e-6, 2, opt=IntegratorOptions(newton_max=1))
    assert np.all(r["status"] == oracle.CELL_NEWTON_FAIL)
    np.testing.assert_array_equal(r["y"], y0)
    assert np.all(r["steps"] == 0)
