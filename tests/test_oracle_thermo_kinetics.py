"""Pins of the oracle's thermodynamics and source terms against facts independent of its code.

* NASA-7 identities dH/dT = Cp, dS/dT = Cp/T, G = H - T S (Table 1) and the constant-cp
  closed form;
* the paper's worked Arrhenius example (Section 4.3) against its closed form in mpmath;
* mass and element conservation of omega (eq. chemical-reaction-mass-conservation);
* detailed balance: at any state whose chemical potentials are a combination of element
  potentials (a Gibbs equilibrium), every rate of progress vanishes -- this fixes the sign
  of ln K and the (p_ref/RT)^(sum nu) factor of eq. equilibrium-constant;
* Troe: F equals F_cent at the centre of the falloff curve (log10 Pr = -c), the paper's
  extreme-parameter case (Appendix C.1), and the low/high pressure limits of eq.
  falloff-reaction;
* the third-body prefactor [M] = sum alpha_i C_i (eq. third_body).
"""

import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from oracle.kinetics import _troe
from oracle.mechanism import Mechanism, R
from synth.states import paper_sampler, sample_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _states(mech, n=64, seed=7):
    T, p, Y = paper_sampler(mech.ns, n, seed)
    return oracle.state_from_TPY(mech, T, p, Y)


def test_nasa7_identities(mech_methane):
    m = mech_methane
    rng = np.random.default_rng(1)
    T = rng.uniform(320.0, 4800.0, size=200)
    T = T[np.abs(T - 1000.0) > 5.0]
    d = 1e-3
    cp, h, s, g = oracle.thermo_mass_specific(m, T)
    _, hp, sp, _ = oracle.thermo_mass_specific(m, T + d)
    _, hm, sm, _ = oracle.thermo_mass_specific(m, T - d)
    np.testing.assert_allclose((hp - hm) / (2 * d), cp, rtol=1e-6, atol=1e-6 * np.abs(h).max())
    np.testing.assert_allclose((sp - sm) / (2 * d), cp / T[:, None], rtol=1e-6)
    np.testing.assert_allclose(g, h - T[:, None] * s, rtol=1e-12, atol=1e-9 * np.abs(h).max())


def test_constant_cp_closed_form():
    doc = json.load(open(os.path.join(GOLDEN, "worked_example_mech.json")))
    for sp in doc["species"]:
        sp["thermo"]["data"] = [[3.5, 0, 0, 0, 0, 1234.0, 5.0], [3.5, 0, 0, 0, 0, 1234.0, 5.0]]
    m = Mechanism(doc)
    T = np.array([300.0, 999.0, 1000.0, 2500.0])
    cp_R, h_RT, s_R, g_RT, dcp = oracle.nasa7_molar(m, T)
    np.testing.assert_allclose(cp_R, 3.5)
    np.testing.assert_allclose(h_RT, np.broadcast_to(3.5 + 1234.0 / T[:, None], h_RT.shape), rtol=1e-15)
    np.testing.assert_allclose(s_R, np.broadcast_to(3.5 * np.log(T)[:, None] + 5.0, s_R.shape), rtol=1e-15)
    np.testing.assert_allclose(dcp, 0.0)


def test_nasa7_range_switch_and_continuity(mech_small):
    m = mech_small
    T = np.array([1000.0 - 1e-9, 1000.0])
    cp_R, h_RT, s_R, _, _ = oracle.nasa7_molar(m, T)
    # the generator makes cp, h and s continuous at the range boundary
    np.testing.assert_allclose(cp_R[0], cp_R[1], rtol=1e-9)
    np.testing.assert_allclose(h_RT[0], h_RT[1], rtol=1e-9)
    np.testing.assert_allclose(s_R[0], s_R[1], rtol=1e-9)
    a = m.nasa_lo[0]
    t = 999.0
    assert oracle.nasa7_molar(m, np.array([t]))[0][0, 0] == pytest.approx(
        a[0] + a[1] * t + a[2] * t**2 + a[3] * t**3 + a[4] * t**4, rel=1e-14)


def test_worked_example_arrhenius():
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["worked_example_reaction"]
    m = Mechanism(json.load(open(os.path.join(GOLDEN, "worked_example_mech.json"))))
    mpmath.mp.dps = 50
    for T in (800.0, 1000.0, 1700.0, 2500.0):
        C = np.array([[0.0, 2e-3, 3e-3, 0.0, 0.0]])
        C[0, 0] = T
        q = oracle.rates_of_progress(m, C)[0][0, 0]
        kf_exact = mpmath.mpf(consts["A"]) * mpmath.power(T, consts["b"]) * mpmath.exp(
            -mpmath.mpf(consts["Ea"]) / (mpmath.mpf("8314.462618") * T))
        exact = kf_exact * mpmath.mpf(2e-3) * mpmath.mpf(3e-3)
        assert abs(q - float(exact)) <= 4e-15 * abs(float(exact))
    # ~4.69e7 m3/kmol/s at 1000 K
    kf1000 = consts["A"] * math.exp(-consts["Ea"] / (R * 1000.0))
    assert kf1000 == pytest.approx(4.69e7, rel=2e-3)


@pytest.mark.parametrize("name", ["h2like_10_27", "ch4like_53_325"])
def test_mass_and_element_conservation(name):
    from synth import mechanism_file
    m = oracle.load_mechanism(mechanism_file(name))
    y = _states(m)
    S = oracle.source_terms(m, y)
    mag = oracle.source_sum_scale(m, y)
    om = S[:, 1:]
    mass = (om * m.W).sum(axis=1)
    assert np.all(np.abs(mass) <= 1e-13 * (mag[:, 1:] * m.W).sum(axis=1))
    for e in range(m.E.shape[0]):
        el = (om * m.E[e]).sum(axis=1)
        assert np.all(np.abs(el) <= 1e-13 * (mag[:, 1:] * m.E[e]).sum(axis=1) + 1e-300)
    # inert species never change
    assert np.all(om[:, m.inert] == 0.0)


@pytest.mark.parametrize("name", ["tiny_8_14", "h2like_10_27", "sri_12_30", "ch4like_53_325"])
def test_detailed_balance_at_gibbs_equilibrium(name):
    """mu_i = g_i + RT ln(C_i RT / p_ref) = sum_e lambda_e E_ei makes every q_j vanish."""
    from synth import mechanism_file
    m = oracle.load_mechanism(mechanism_file(name))
    rng = np.random.default_rng(3)
    for T in (700.0, 1200.0, 2100.0, 3100.0):
        _, _, _, g_RT, _ = oracle.nasa7_molar(m, np.array([T]))
        lam = rng.uniform(-25.0, -5.0, size=m.E.shape[0])
        lnC = np.log(m.p_ref / (R * T)) - g_RT[0] + lam @ m.E
        # shift every element potential by the same s (still an equilibrium) so that max ln C = -2
        n_atoms = m.E.sum(axis=0)
        s = np.max((lnC + 2.0) / n_atoms)
        lnC = lnC - s * n_atoms
        assert lnC.min() > -700.0
        y = np.concatenate([[T], np.exp(lnC)])[None]
        q, Rf, Rr, _ = oracle.rates_of_progress(m, y)
        scale = np.maximum(np.abs(Rf), np.abs(Rr))
        mask = scale > 1e-280
        assert np.all(np.abs(q[mask]) <= 1e-10 * scale[mask]), (name, T, np.max(np.abs(q[mask]) / scale[mask]))


def test_troe_centre_and_extremes():
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))

    class Rx:
        pass
    rx = Rx()
    for alpha, T3, T1, T2 in [(0.6, 150.0, 900.0, 4000.0), (0.45, 2000.0, 60.0, None)]:
        rx.troe = (alpha, T3, T1, T2)
        T = np.array([900.0, 1500.0, 2200.0])
        Fc = (1 - alpha) * np.exp(-T / T3) + alpha * np.exp(-T / T1) + (np.exp(-T2 / T) if T2 else 0.0)
        c = -0.4 - 0.67 * np.log10(Fc)
        Pr_centre = 10.0 ** (-c)
        F, _, _ = _troe(rx, T, Pr_centre)
        np.testing.assert_allclose(F, Fc, rtol=1e-13)
        # far from the centre F -> 1 (both limits) only as fast as f1 grows; check monotone trend
        Fh, _, _ = _troe(rx, T, Pr_centre * 1e30)
        assert np.all(np.abs(np.log(Fh)) < np.abs(np.log(Fc)))
    # paper's extreme case: T3 -> 0 kills term 1, T1 -> infinity makes term 2 alpha, no T2
    ex = consts["troe_extreme"]
    rx.troe = (0.7, ex["T3"], ex["T1"], None)
    T = np.array([1000.0, 2000.0])
    F, _, _ = _troe(rx, T, np.array([10.0 ** 0.5, 10.0 ** 0.5]))
    L = math.log10(0.7)
    x = 0.5 - 0.4 - 0.67 * L
    f1 = x / (0.75 - 1.27 * L - 0.14 * x)
    np.testing.assert_allclose(F, 10.0 ** (L / (1 + f1 * f1)), rtol=1e-14)


def test_falloff_limits_and_third_body():
    doc = json.load(open(os.path.join(GOLDEN, "worked_example_mech.json")))
    base = doc["reactions"][0]
    doc["reactions"] = [
        dict(base, type="falloff", **{"high-P-rate-constant": {"A": 2e10, "b": 0.3, "Ea": 1e7},
                                       "low-P-rate-constant": {"A": 5e12, "b": -0.7, "Ea": 2e6}}),
        dict(base, type="three-body", efficiencies={"O": 3.0}),
    ]
    for r in doc["reactions"]:
        r.pop("rate-constant", None) if r["type"] == "falloff" else None
    doc["reactions"][1]["rate-constant"] = {"A": 3e9, "b": 0.5, "Ea": 5e6}
    m = Mechanism(doc)
    T = 1300.0
    kinf = 2e10 * T**0.3 * math.exp(-1e7 / (R * T))
    k0 = 5e12 * T**-0.7 * math.exp(-2e6 / (R * T))
    kA = 3e9 * T**0.5 * math.exp(-5e6 / (R * T))
    for Mtot in (1e-9, 1e9):
        C = np.array([[T, 0.2 * Mtot, 0.3 * Mtot, 0.1 * Mtot, 0.4 * Mtot]])
        q, Rf, _, _ = oracle.rates_of_progress(m, C)
        kf_fo = Rf[0, 0] / (C[0, 1] * C[0, 2])
        Mc = C[0, 1:].sum()
        if Mtot < 1:     # low pressure: k_f -> k0 [M]
            assert kf_fo == pytest.approx(k0 * Mc, rel=1e-6)
        else:            # high pressure: k_f -> k_inf
            assert kf_fo == pytest.approx(kinf, rel=1e-6)
        Meff = Mc + 2.0 * C[0, 3]
        assert Rf[0, 1] == pytest.approx(kA * Meff * C[0, 1] * C[0, 2], rel=1e-13)


def test_source_terms_state_shapes(mech_small):
    T, p, Y = sample_config("be_small", mech_small.ns, 5)
    y = oracle.state_from_TPY(mech_small, T, p, Y)
    # the init map reproduces the ideal-gas pressure and the mass fractions
    np.testing.assert_allclose(R * T * y[:, 1:].sum(axis=1), p, rtol=1e-14)
    np.testing.assert_allclose(oracle.mass_fractions(mech_small, y), Y, rtol=1e-13, atol=1e-16)
    S = oracle.source_terms(mech_small, y)
    assert S.shape == (5, mech_small.n) and np.all(np.isfinite(S))
