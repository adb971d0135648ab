"""Pins of the oracle's integrators (Section 3.2, Appendix A) against independent facts.

* a linear isomerisation A <=> B with equal enthalpies (T stays constant, dC/dt = K C):
  backward Euler must equal (I - hK)^-N exactly, and both schemes converge to expm(K t)
  at orders 1 and 2;
* convergence order on a synthetic mechanism (the study of Section 5.4);
* linear invariants (element totals, mass) are kept by every Newton iterate and
  Rosenbrock stage; the constant-pressure invariant rho*h drifts at the scheme's order;
* a long integration relaxes to a Gibbs equilibrium (every q_j -> 0, detailed balance);
* the per-cell failure statuses.
"""

import json
import os

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle.integrate import IntegratorOptions
from oracle.mechanism import Mechanism, R
from synth.states import sample_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _isomer_mech():
    doc = json.load(open(os.path.join(GOLDEN, "worked_example_mech.json")))
    a = [3.1, 1.2e-3, -3.0e-7, 4.0e-11, -2.0e-15, -1.2e4, 4.0]
    sp = doc["species"][:3]
    sp[0] = dict(sp[0], name="A", composition={"O": 2}, **{"molecular-weight": 31.998})
    sp[1] = dict(sp[1], name="B", composition={"O": 2}, **{"molecular-weight": 31.998})
    sp[2] = dict(sp[2], name="N", composition={"O": 1}, **{"molecular-weight": 15.999})
    sp[0]["thermo"] = {"model": "NASA7", "temperature-ranges": [300, 1000, 5000], "data": [a, a]}
    b = list(a)
    b[6] = a[6] + 1.3           # B differs from A only by its entropy constant
    sp[1]["thermo"] = {"model": "NASA7", "temperature-ranges": [300, 1000, 5000], "data": [b, b]}
    sp[2]["thermo"] = {"model": "NASA7", "temperature-ranges": [300, 1000, 5000], "data": [a, a]}
    doc["species"] = sp
    doc["reactions"] = [{"equation": "A <=> B", "type": "elementary", "reversible": True,
                         "reactants": {"A": 1}, "products": {"B": 1},
                         "rate-constant": {"A": 3e9, "b": 0.0, "Ea": 1.2e8}}]
    return Mechanism(doc)


def _linear_K(m, T):
    kf = 3e9 * np.exp(-1.2e8 / (R * T))
    Kc = np.exp(1.3)            # -dG/RT = (s_B - s_A)/R, sum nu = 0
    kr = kf / Kc
    return np.array([[-kf, kr, 0.0], [kf, -kr, 0.0], [0.0, 0.0, 0.0]])


def test_linear_isomerisation_be_exact_and_orders():
    m = _isomer_mech()
    T = 1400.0
    y0 = np.array([[T, 0.006, 0.001, 0.002]])
    K = _linear_K(m, T)
    tend = 0.5 / abs(K[0, 0])
    exact = expm(K * tend) @ y0[0, 1:]
    errs_be, errs_ros = [], []
    for N in (8, 16, 32, 64):
        h = tend / N
        r = oracle.integrate_be(m, y0, tend, N)
        assert r["status"][0] == 0
        np.testing.assert_allclose(r["y"][0, 0], T, rtol=0, atol=1e-9)
        ref = np.linalg.matrix_power(np.linalg.inv(np.eye(3) - h * K), N) @ y0[0, 1:]
        np.testing.assert_allclose(r["y"][0, 1:], ref, rtol=1e-12, atol=1e-18)
        errs_be.append(np.abs(r["y"][0, 1:] - exact).max())
        r2 = oracle.integrate_ros2(m, y0, tend, fixed_steps=N)
        errs_ros.append(np.abs(r2["y"][0, 1:] - exact).max())
    o_be = np.log2(np.array(errs_be[:-1]) / np.array(errs_be[1:]))
    o_ros = np.log2(np.array(errs_ros[:-1]) / np.array(errs_ros[1:]))
    assert np.all(np.abs(o_be - 1.0) < 0.2) and abs(o_be[-1] - 1.0) < 0.1, o_be
    assert np.all(np.abs(o_ros - 2.0) < 0.2) and abs(o_ros[-1] - 2.0) < 0.1, o_ros
    # the adaptive controller meets its tolerance on the same problem
    r3 = oracle.integrate_ros2(m, y0, tend, opt=IntegratorOptions(rtol=1e-8, atol=1e-14))
    Y3 = r3["y"][0, 1:] * m.W / (r3["y"][0, 1:] * m.W).sum()
    Ye = exact * m.W / (exact * m.W).sum()
    assert np.abs(Y3 - Ye).max() < 1e-6


def _onto_manifold(m, n=2, t=2e-7):
    T, p, Y = sample_config("be_small", m.ns, n)
    y = oracle.state_from_TPY(m, T, p, Y)
    return oracle.integrate_ros2(m, y, t)["y"]


def test_convergence_orders_on_mechanism(mech_small):
    m = mech_small
    y0 = _onto_manifold(m)
    t = 2e-9
    ref = oracle.integrate_ros2(m, y0, t, fixed_steps=512)["y"]
    e_be, e_ro = [], []
    for N in (16, 32, 64, 128):
        e_be.append(np.abs(oracle.integrate_be(m, y0, t, N)["y"][:, 1:] - ref[:, 1:]).max())
        e_ro.append(np.abs(oracle.integrate_ros2(m, y0, t, fixed_steps=N)["y"][:, 1:] - ref[:, 1:]).max())
    o_be = np.log2(np.array(e_be[:-1]) / np.array(e_be[1:]))
    o_ro = np.log2(np.array(e_ro[:-1]) / np.array(e_ro[1:]))
    assert np.median(o_be) == pytest.approx(1.0, abs=0.25), o_be
    assert np.median(o_ro) == pytest.approx(2.0, abs=0.3), o_ro


def _enthalpy_density(m, y):
    _, h_RT, _, _, _ = oracle.nasa7_molar(m, y[:, 0])
    return (y[:, 1:] * h_RT * R * y[:, 0][:, None]).sum(axis=1)


def test_invariants(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 6)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    el0 = y0[:, 1:] @ m.E.T
    mass0 = y0[:, 1:] @ m.W
    for r in (oracle.integrate_be(m, y0, 2e-6, 20), oracle.integrate_ros2(m, y0, 2e-7)):
        y = r["y"]
        np.testing.assert_allclose(y[:, 1:] @ m.E.T, el0, rtol=1e-11)
        np.testing.assert_allclose(y[:, 1:] @ m.W, mass0, rtol=1e-12)
        np.testing.assert_allclose(y[:, 1 + np.nonzero(m.inert)[0]], y0[:, 1 + np.nonzero(m.inert)[0]], rtol=1e-13)
    # rho*h is conserved by the constant-pressure ODE; the schemes keep it to their order
    y1 = _onto_manifold(m, 2)
    H0 = _enthalpy_density(m, y1)
    t = 2e-9
    d_be, d_ro = [], []
    for N in (16, 32, 64):
        d_be.append(np.abs(_enthalpy_density(m, oracle.integrate_be(m, y1, t, N)["y"]) - H0).max())
        d_ro.append(np.abs(_enthalpy_density(m, oracle.integrate_ros2(m, y1, t, fixed_steps=N)["y"]) - H0).max())
    assert d_be[-1] < d_be[0] / 2.5
    assert d_ro[-1] < d_ro[0] / 6.0


def test_relaxation_to_equilibrium(mech_tiny):
    m = mech_tiny
    T, p, Y = sample_config("be_small", m.ns, 3)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    # backward Euler is L-stable: with growing steps it walks to the steady state
    y = y0
    for k in range(16):
        r = oracle.integrate_be(m, y, 10.0 ** (k - 9), 10)
        assert np.all(r["status"] == 0)
        y = r["y"]
    r = {"y": y}
    q, Rf, Rr, _ = oracle.rates_of_progress(m, r["y"])
    scale = np.maximum(np.abs(Rf), np.abs(Rr))
    live = scale > 1e-200
    ratio = np.abs(q[live]) / scale[live]
    assert ratio.max() <= 1e-8, ratio.max()
    # far from equilibrium the same ratios are of order one
    q0, Rf0, Rr0, _ = oracle.rates_of_progress(m, y0)
    assert np.max(np.abs(q0) / np.maximum(np.abs(Rf0), np.abs(Rr0))) > 0.5
    # the equilibrium keeps the linear invariants of the initial state (rho*h is kept only to
    # the O(dt) accuracy of the large backward-Euler steps, so it is not checked here)
    np.testing.assert_allclose(r["y"][:, 1:] @ m.E.T, y0[:, 1:] @ m.E.T, rtol=1e-10)


def test_failure_statuses(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 4)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    bad = y0.copy()
    bad[0, 3] = np.nan
    bad[1, 0] = -5.0
    r = oracle.integrate_be(m, bad, 1e-7, 2)
    assert list(r["status"][:2]) == [oracle.CELL_NONFINITE, oracle.CELL_T_RANGE]
    np.testing.assert_array_equal(r["y"][1], bad[1])
    r = oracle.integrate_ros2(m, bad, 1e-8)
    assert list(r["status"][:2]) == [oracle.CELL_NONFINITE, oracle.CELL_T_RANGE]
    # Newton limited to one iteration and no halving: every cell fails
    r = oracle.integrate_be(m, y0, 1e-6, 1, opt=IntegratorOptions(newton_max=1, halving_max_depth=0))
    assert np.all(r["status"] == oracle.CELL_NEWTON_FAIL)
    np.testing.assert_array_equal(r["y"], y0)
    # a floor on h above the first rejected step: DT_UNDERFLOW
    r = oracle.integrate_ros2(m, y0, 1e-6, opt=IntegratorOptions(h_min=1e-7))
    assert np.all(np.isin(r["status"], [oracle.CELL_DT_UNDERFLOW, oracle.CELL_OK]))
    assert np.any(r["status"] == oracle.CELL_DT_UNDERFLOW)
    r = oracle.integrate_ros2(m, y0, 1e-6, opt=IntegratorOptions(max_steps=3))
    assert np.all(r["status"] == oracle.CELL_MAX_STEPS)
    assert np.all(r["accepted"] + r["rejected"] == 3)
