"""Pins of the oracle's backward-Euler sensitivities.

* the tangent (forward sensitivity) against central finite differences of the forward map
  (h = 1e-6 in ln A and relative 1e-6 in the initial state);
* the adjoint against the tangent (the dot-product identity lambda_N . s_N = g);
* the init-map and loss pull-backs against finite differences.
"""

import numpy as np

import oracle
from oracle.sensitivity import be_adjoint, be_tangent, final_loss, init_map_vjp
from synth.states import loss_weights, sample_config

DT, NSTEPS = 1e-7, 12


def _setup(m, n=3):
    T, p, Y = sample_config("be_small", m.ns, n)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    return T, p, Y, y0


def _forward(m, y0, lnA=None):
    return oracle.integrate_be(m, y0, DT, NSTEPS, lnA=lnA, record=True)


def test_tangent_matches_central_differences(mech_tiny):
    m = mech_tiny
    _, _, _, y0 = _setup(m)
    r = _forward(m, y0)
    assert np.all(r["status"] == 0)
    s = be_tangent(m, y0, r["trajectory"])
    h = 1e-6
    for j in range(m.nr):
        lp = m.lnA_default.copy()
        lm = m.lnA_default.copy()
        lp[j] += h
        lm[j] -= h
        fd = (_forward(m, y0, lp)["y"] - _forward(m, y0, lm)["y"]) / (2 * h)
        scale = np.abs(s[:, :, j]).max(axis=1, keepdims=True)
        noise = 1e-15 * np.abs(r["y"]) / h        # differences below rounding of y_N
        assert np.all(np.abs(fd - s[:, :, j]) <= 1e-5 * scale + noise), j
    for k in range(m.n):
        d = 1e-6 * np.abs(y0[:, k]).max()
        yp = y0.copy()
        ym = y0.copy()
        yp[:, k] += d
        ym[:, k] -= d
        fd = (_forward(m, yp)["y"] - _forward(m, ym)["y"]) / (2 * d)
        col = s[:, :, m.nr + k]
        scale = np.abs(col).max(axis=1, keepdims=True)
        noise = 1e-15 * np.abs(r["y"]) / d
        assert np.all(np.abs(fd - col) <= 1e-5 * scale + noise), k


def test_adjoint_matches_tangent(mech_small):
    m = mech_small
    T, p, Y, y0 = _setup(m, 4)
    r = _forward(m, y0)
    w = loss_weights(y0.shape[0], m.ns)
    L, lam = final_loss(m, r["y"], w)
    s = be_tangent(m, y0, r["trajectory"])
    lam0, g = be_adjoint(m, lam, r["trajectory"])
    via_tangent = np.einsum("ci,cik->ck", lam, s)
    np.testing.assert_allclose(g, via_tangent[:, :m.nr], rtol=1e-9, atol=1e-12 * np.abs(g).max())
    np.testing.assert_allclose(lam0, via_tangent[:, m.nr:], rtol=1e-9, atol=1e-12 * np.abs(lam0).max())


def test_loss_and_init_map_pullbacks(mech_small):
    m = mech_small
    T, p, Y, y0 = _setup(m, 3)
    w = loss_weights(3, m.ns)
    L, lam = final_loss(m, y0, w)
    for k in range(m.n):
        d = 1e-4 * np.abs(y0[:, k]).max()
        yp = y0.copy()
        ym = y0.copy()
        yp[:, k] += d
        ym[:, k] -= d
        fd = (final_loss(m, yp, w)[0] - final_loss(m, ym, w)[0]) / (2 * d)
        assert abs(fd - lam[:, k].sum()) <= 1e-6 * np.abs(lam[:, k]).sum() + 1e-12
    rng = np.random.default_rng(2)
    lam0 = rng.standard_normal(y0.shape)
    dT, dY = init_map_vjp(m, T, p, Y, lam0)
    f = lambda TT, YY: (oracle.state_from_TPY(m, TT, p, YY) * lam0).sum()  # noqa: E731
    d = 1e-4
    assert abs((f(T + d, Y) - f(T - d, Y)) / (2 * d) - dT.sum()) <= 1e-6 * np.abs(dT).sum()
    fC = lambda YY: (oracle.state_from_TPY(m, T, p, YY)[:, 1:] * lam0[:, 1:]).sum()  # noqa: E731
    for k in range(m.ns):
        Yp = Y.copy()
        Ym = Y.copy()
        Yp[:, k] += 1e-7
        Ym[:, k] -= 1e-7
        fd = (fC(Yp) - fC(Ym)) / 2e-7
        assert abs(fd - dY[:, k].sum()) <= 1e-6 * np.abs(dY[:, k]).sum() + 1e-9
