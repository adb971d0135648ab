"""Pins of the oracle's P-log rates (Section 2.2, other pressure-dependent forms) by closed forms:

* at a tabulated pressure (p = R T sum C placed on it) k equals that set's Arrhenius rate;
* below the lowest and above the highest pressure k equals the end sets;
* at the geometric mean of two neighbouring pressures ln k is the mean of their ln k;
* a one-entry table behaves as the elementary reaction with the same parameters;
* the analytic Jacobian equals the complex-step Jacobian at pressures that cover every interval and
  both clamps (the dependence on every concentration through p included), in both energy modes.
"""

import json
import math

import numpy as np
import pytest

import oracle
from oracle.kinetics import _forward_rate
from oracle.mechanism import R, Mechanism
from synth import mechanism_file
from synth.states import sample_config


def _doc():
    return json.load(open(mechanism_file("plog_12_30")))


def _states_at(m, p, n=None):
    n = len(p) if n is None else n
    T, _, Y = sample_config("ros2_1m", m.ns, n)
    return oracle.state_from_TPY(m, T, np.asarray(p, dtype=float), Y)


def _arrhenius(k, T):
    return k["A"] * T ** k["b"] * np.exp(-k["Ea"] / (R * T))


def _plog_reactions(m, doc):
    return [(j, r) for j, r in enumerate(doc["reactions"]) if r["type"] == "pressure-dependent-Arrhenius"]


def test_tabulated_pressures_and_clamps():
    doc = _doc()
    m = Mechanism(doc)
    table = _plog_reactions(m, doc)
    assert len(table) == 8
    pressures = sorted(k["P"] for k in table[0][1]["rate-constants"])
    for p, which in [(pressures[0], 0), (pressures[1], 1), (pressures[2], 2),
                     (pressures[0] / 7.0, 0), (pressures[2] * 5.0, 2)]:
        y = _states_at(m, [p] * 6)
        T, C = y[:, 0], y[:, 1:]
        for j, r in table:
            ks = sorted(r["rate-constants"], key=lambda k: k["P"])
            kf = _forward_rate(m, m.reactions[j], j, T, np.log(T), 1.0 / T, C, m.lnA_default)[0]
            np.testing.assert_allclose(kf, _arrhenius(ks[which], T), rtol=1e-12)


def test_log_linear_between_pressures():
    doc = _doc()
    m = Mechanism(doc)
    for j, r in _plog_reactions(m, doc):
        ks = sorted(r["rate-constants"], key=lambda k: k["P"])
        for i in range(2):
            pm = math.sqrt(ks[i]["P"] * ks[i + 1]["P"])
            y = _states_at(m, [pm] * 5)
            T, C = y[:, 0], y[:, 1:]
            kf = _forward_rate(m, m.reactions[j], j, T, np.log(T), 1.0 / T, C, m.lnA_default)[0]
            ref = np.sqrt(_arrhenius(ks[i], T) * _arrhenius(ks[i + 1], T))
            np.testing.assert_allclose(kf, ref, rtol=1e-10)


def test_single_entry_table_is_elementary():
    doc = _doc()
    j, r = _plog_reactions(Mechanism(doc), doc)[0]
    k = r["rate-constants"][1]
    one = json.loads(json.dumps(doc))
    one["reactions"][j]["rate-constants"] = [k]
    elem = json.loads(json.dumps(doc))
    elem["reactions"][j] = {kk: v for kk, v in r.items() if kk != "rate-constants"}
    elem["reactions"][j]["type"] = "elementary"
    elem["reactions"][j]["rate-constant"] = {"A": k["A"], "b": k["b"], "Ea": k["Ea"]}
    m1, me = Mechanism(one), Mechanism(elem)
    y = _states_at(m1, np.geomspace(1e3, 1e7, 9))
    np.testing.assert_allclose(oracle.source_terms(m1, y), oracle.source_terms(me, y), rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("energy", [0, 1])
def test_jacobian_complex_step_over_pressures(energy):
    m = oracle.load_mechanism(mechanism_file("plog_12_30"))
    y = _states_at(m, np.geomspace(3e3, 3e6, 40))
    J, M = oracle.jacobian(m, y, energy=energy, magnitude=True)
    Jc = oracle.jacobian_complex_step(m, y, energy=energy)
    assert np.all(np.abs(J - Jc) <= 1e-11 * (np.abs(Jc) + M))
    # the p-dependence reaches inert species' columns too
    inert = 1 + np.nonzero(m.inert)[0]
    assert np.abs(Jc[:, :, inert]).max() > 0.0
