"""Pins of the oracle's SRI falloff broadening (Section 2.2, SRI broadening), by reduction to cases
fixed without the SRI formula:

* a = 0, c -> inf, d = 1, e = 0 makes the bracket 1 and F = 1: the Lindemann rate;
* with a = 0 and c -> inf the bracket stays 1, so F = d T^e exactly: k_f = d T^e k_f(Lindemann);
* F is proportional to d for any a, b, c, e: doubling d doubles k_f.
The analytic derivatives are pinned by the complex-step Jacobian test on the SRI mechanism.
"""

import json

import numpy as np
import pytest

import oracle
from oracle.kinetics import _forward_rate
from oracle.mechanism import Mechanism
from synth import mechanism_file
from synth.states import sample_config


def _mech(sri):
    doc = json.load(open(mechanism_file("sri_12_30")))
    for r in doc["reactions"]:
        if "SRI" in r:
            if sri is None:
                del r["SRI"]
            else:
                r["SRI"] = dict(sri) if isinstance(sri, dict) else sri(r["SRI"])
    return Mechanism(doc)


def _kf(m):
    T, p, Y = sample_config("ros2_1m", m.ns, 16)
    y = oracle.state_from_TPY(m, T, p, Y)
    T, C = y[:, 0], y[:, 1:]
    out = []
    for j, rx in enumerate(m.reactions):
        if rx.kind == "falloff":
            out.append(_forward_rate(m, rx, j, T, np.log(T), 1.0 / T, C, m.lnA_default)[0])
    return np.array(out), T


def test_sri_mechanism_has_sri_falloff():
    m = _mech(lambda s: s)
    assert sum(rx.sri is not None for rx in m.reactions) == 6


def test_sri_reduces_to_lindemann():
    k_lind, _ = _kf(_mech(None))
    k_sri, _ = _kf(_mech({"A": 0.0, "B": 300.0, "C": 1e300, "D": 1.0, "E": 0.0}))
    np.testing.assert_allclose(k_sri, k_lind, rtol=1e-14)


@pytest.mark.parametrize("e", [-0.4, 0.7])
def test_sri_power_of_T(e):
    k_lind, T = _kf(_mech(None))
    k_sri, _ = _kf(_mech({"A": 0.0, "B": 300.0, "C": 1e300, "D": 1.3, "E": e}))
    np.testing.assert_allclose(k_sri, 1.3 * T[None, :] ** e * k_lind, rtol=1e-13)


def test_sri_proportional_to_d():
    k1, _ = _kf(_mech(lambda s: dict(s, D=1.0)))
    k2, _ = _kf(_mech(lambda s: dict(s, D=2.0)))
    np.testing.assert_allclose(k2, 2.0 * k1, rtol=1e-14)
    k0, _ = _kf(_mech(None))
    assert np.max(np.abs(k1 / k0 - 1.0)) > 1e-3          # the broadening is active
