"""Pins of the oracle's Rosenbrock discrete adjoint (the reverse sweep along a fixed step sequence).

* the frozen-step replay reproduces the adaptive integration it was recorded from;
* dL/dlnA and dL/dy0 of L = w . y_N equal complex-step derivatives of the replayed forward map
  (exact to rounding: the whole Rosenbrock step, including the dependence of its iteration
  matrix on the state, is carried in complex arithmetic), in both energy modes, at adaptive
  steps and at fixed steps large enough for the second-derivative terms to matter;
* the same derivatives agree with central finite differences (h = 1e-6);
* the pin is sensitive: an adjoint without the second-derivative terms (J'(y)[g] and
  (dS/dlnA)'(y)[g]) misses the complex-step values by far more than the tolerance.
"""

import numpy as np
import pytest

import oracle
import oracle.sensitivity as sens
from oracle.sensitivity import ros2_adjoint, ros2_adjoint_cell, ros2_replay
from synth.states import sample_config

DT = 1e-9          # adaptive: 1 to 15 accepted steps per cell for these states
CS_H = 1e-40
# fixed steps of 2e-8 s: large enough that the second-derivative terms change the result by
# 0.2 - 9 % (at the adaptive steps above they are 1e-8 - 5e-6 of it)
FIXED = (1e-7, 5)


def _setup(m, n=4, energy=0, fixed=False):
    T, p, Y = sample_config("ros2_1m", m.ns, n)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    opt = oracle.IntegratorOptions(energy=energy)
    if fixed:
        r = oracle.integrate_ros2(m, y0, FIXED[0], opt=opt, record=True, fixed_steps=FIXED[1])
    else:
        r = oracle.integrate_ros2(m, y0, DT, opt=opt, record=True)
    assert np.all(r["status"] == 0)
    steps = [[h for h, _ in hist] for hist in r["history"]]
    return y0, r, steps


def _weights(m, yN, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(m.n) / np.maximum(np.abs(yN), 1e-12)


def test_replay_reproduces_integration(mech_small):
    m = mech_small
    y0, r, steps = _setup(m)
    for c in range(len(steps)):
        yN = ros2_replay(m, y0[c], steps[c])
        assert np.all(np.abs(yN - r["y"][c]) <= 1e-13 * np.abs(r["y"][c]) + 1e-300)


@pytest.mark.parametrize("energy,fixed", [(0, False), (1, False), (0, True), (1, True)])
def test_adjoint_matches_complex_step(mech_small, energy, fixed):
    m = mech_small
    y0, r, steps = _setup(m, energy=energy, fixed=fixed)
    for c in (0, 3):
        w = _weights(m, r["y"][c], 10 + c)
        lam0, g = ros2_adjoint_cell(m, w, y0[c], steps[c], energy=energy)
        g_cs = np.zeros(m.nr)
        for j in range(m.nr):
            lnA = m.lnA_default.astype(complex)
            lnA[j] += 1j * CS_H
            g_cs[j] = np.imag(w @ ros2_replay(m, y0[c], steps[c], lnA, energy)) / CS_H
        lam_cs = np.zeros(m.n)
        for k in range(m.n):
            yc = y0[c].astype(complex)
            yc[k] += 1j * CS_H
            lam_cs[k] = np.imag(w @ ros2_replay(m, yc, steps[c], None, energy)) / CS_H
        assert np.max(np.abs(g - g_cs)) <= 1e-10 * np.max(np.abs(g_cs)), c
        # per component, relative to the component's own size (T and C differ by ~1e7)
        assert np.all(np.abs(lam0 - lam_cs) <= 1e-10 * np.abs(lam_cs) + 1e-12 * np.max(np.abs(lam_cs))), c


@pytest.mark.parametrize("fixed", [False, True])
def test_adjoint_matches_central_differences(mech_small, fixed):
    m = mech_small
    y0, r, steps = _setup(m, n=2, fixed=fixed)
    c = 0
    w = _weights(m, r["y"][c], 3)
    lam0, g = ros2_adjoint_cell(m, w, y0[c], steps[c])
    h = 1e-6
    for j in range(0, m.nr, 3):
        lp, lm = m.lnA_default.copy(), m.lnA_default.copy()
        lp[j] += h
        lm[j] -= h
        fd = (w @ ros2_replay(m, y0[c], steps[c], lp) - w @ ros2_replay(m, y0[c], steps[c], lm)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * np.max(np.abs(g)), j
    for k in range(m.n):
        d = 1e-6 * abs(y0[c, k])
        yp, ym = y0[c].copy(), y0[c].copy()
        yp[k] += d
        ym[k] -= d
        fd = (w @ ros2_replay(m, yp, steps[c]) - w @ ros2_replay(m, ym, steps[c])) / (2 * d)
        assert abs(fd - lam0[k]) <= 1e-5 * abs(lam0[k]) + 1e-9 * np.max(np.abs(lam0 * y0[c])) / abs(y0[c, k]), k


def test_per_cell_driver_matches_single_cell(mech_small):
    m = mech_small
    y0, r, steps = _setup(m, n=3)
    lam_N = np.stack([_weights(m, r["y"][c], c) for c in range(3)])
    lam0, g = ros2_adjoint(m, lam_N, y0, r["history"])
    for c in range(3):
        l1, g1 = ros2_adjoint_cell(m, lam_N[c], y0[c], steps[c])
        np.testing.assert_array_equal(lam0[c], l1)
        np.testing.assert_array_equal(g[c], g1)


def test_dropping_second_derivative_terms_is_detected(mech_small, monkeypatch):
    m = mech_small
    y0, r, steps = _setup(m, fixed=True)
    c = 2
    w = _weights(m, r["y"][c], 7)
    g_cs = np.zeros(m.nr)
    for j in range(m.nr):
        lnA = m.lnA_default.astype(complex)
        lnA[j] += 1j * CS_H
        g_cs[j] = np.imag(w @ ros2_replay(m, y0[c], steps[c], lnA)) / CS_H
    monkeypatch.setattr(sens, "_directional", lambda f, y, v: np.zeros_like(f(y[None, :])[0]))
    _, g_bad = ros2_adjoint_cell(m, w, y0[c], steps[c])
    assert np.max(np.abs(g_bad - g_cs)) > 1e-4 * np.max(np.abs(g_cs))
