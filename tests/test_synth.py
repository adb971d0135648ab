"""The seeded input generators: deterministic, element-balanced, full stoichiometric rank."""

import json

import numpy as np
import pytest

from synth import generate_mechanism, MECH_CONFIGS
from synth.states import sample_states


@pytest.mark.parametrize("name", ["tiny_5_6", "tiny_8_14", "h2like_10_27", "sri_12_30", "plog_12_30", "mix_30_90", "ch4like_53_325"])
def test_mechanism_structure(name):
    doc = generate_mechanism(name)
    cfg = MECH_CONFIGS[name]
    assert json.dumps(doc) == json.dumps(generate_mechanism(name))   # deterministic
    sp = {s["name"]: s for s in doc["species"]}
    assert len(sp) == cfg.n_species and len(doc["reactions"]) == cfg.n_reactions
    kinds = [r["type"] for r in doc["reactions"]]
    assert kinds.count("three-body") == cfg.n_third_body and kinds.count("falloff") == cfg.n_falloff
    names = list(sp)
    nu = np.zeros((len(names), len(doc["reactions"])))
    for j, r in enumerate(doc["reactions"]):
        assert 1 <= sum(r["reactants"].values()) <= 3 and 1 <= sum(r["products"].values()) <= 3
        for el in [e["symbol"] for e in doc["elements"]]:
            lhs = sum(c * sp[s]["composition"].get(el, 0) for s, c in r["reactants"].items())
            rhs = sum(c * sp[s]["composition"].get(el, 0) for s, c in r["products"].items())
            assert lhs == rhs
        for s, c in r["reactants"].items():
            nu[names.index(s), j] -= c
            assert not sp[s]["inert"]
        for s, c in r["products"].items():
            nu[names.index(s), j] += c
    assert np.linalg.matrix_rank(nu) == doc["generator"]["stoichiometric-rank"]
    for s in doc["species"]:
        lo, hi = s["thermo"]["data"]
        t = 1000.0
        cp = lambda a: sum(a[k] * t ** k for k in range(5))  # noqa: E731
        assert cp(lo) == pytest.approx(cp(hi), rel=1e-10)


def test_states_reproducible_and_normalised():
    T, p, Y = sample_states(10, 100, 2000, (1000.0, 1500.0), 1.0)
    T2, _, Y2 = sample_states(10, 40, 2000, (1000.0, 1500.0), 1.0, first=60)
    np.testing.assert_array_equal(T[60:], T2)
    np.testing.assert_array_equal(Y[60:], Y2)
    np.testing.assert_allclose(Y.sum(axis=1), 1.0, rtol=1e-14)
    assert T.min() >= 1000.0 and T.max() <= 1500.0 and np.all(p == 101325.0)
