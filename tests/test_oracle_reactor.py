"""Pins of the oracle's constant-pressure reactor form (energy CONST_P_REACTOR).

The reactor keeps p fixed, so the density follows T and the mole number (the paper's
constant-pressure source terms of Appendix B hold the density instead).  Its sources in (T, C)
are pinned by routes that do not use the dilatation formula:

* the chain rule through the mass-fraction form: with Y and p held by the state, C(T, Y) =
  p/(R T) (Y_i/W_i) / sum_j Y_j/W_j, dY_i/dt = W_i omega_i / rho and dT/dt = omega_T; the
  directional derivative of C(T, Y) along (dT/dt, dY/dt) (complex step, exact to rounding) must
  equal the species sources;
* its rates of change of p = R T sum C and of the mass-specific enthalpy vanish;
* a thermoneutral, mole-conserving reaction (A <=> B with equal enthalpies) has g = 0, so the
  reactor form equals the constant-pressure form;
* the analytic Jacobian and d/d ln A against complex-step derivatives of the sources;
* integration: the oracle's backward Euler and Rosenbrock converge to an independent stiff
  solution (scipy's Radau) of the mass-fraction ODE, at order 1 for backward Euler.
"""

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import CONST_P, CONST_P_REACTOR
from oracle.integrate import IntegratorOptions
from oracle.mechanism import R
from synth import mechanism_file
from synth.states import paper_sampler, sample_config

MECHS = ["tiny_8_14", "h2like_10_27", "sri_12_30", "plog_12_30", "mix_30_90"]


def _mech(name):
    return oracle.load_mechanism(mechanism_file(name))


def _states(m, n, seed=31):
    T, p, Y = paper_sampler(m.ns, n, seed)
    keep = np.abs(T - 1000.0) > 150.0   # clear of the NASA range switch for complex steps in T
    return oracle.state_from_TPY(m, T[keep], p[keep], Y[keep])


def _conc(m, T, Y, p):
    """C(T, Y) at pressure p (complex-safe): p/(R T) times the mole fractions."""
    z = Y / m.W[None, :]
    return (p / (R * T))[:, None] * z / z.sum(axis=1)[:, None]


def _mass_fraction_rhs(m, T, Y, p, lnA=None):
    """(dT/dt, dY/dt) of the reactor in (T, Y): the paper's omega and constant-pressure omega_T."""
    C = _conc(m, T, Y, p)
    y = np.concatenate([T[:, None], C], axis=1)
    S0 = oracle.source_terms(m, y, lnA, CONST_P)
    rho = (C * m.W[None, :]).sum(axis=1)
    return S0[:, 0], S0[:, 1:] * m.W[None, :] / rho[:, None]


def _to_TYp(m, y):
    T, C = y[:, 0], y[:, 1:]
    rho = (C * m.W[None, :]).sum(axis=1)
    return T, C * m.W[None, :] / rho[:, None], R * T * C.sum(axis=1)


@pytest.mark.parametrize("name", MECHS)
def test_sources_are_the_chain_rule_of_the_mass_fraction_form(name):
    m = _mech(name)
    y = _states(m, 24)
    T, Y, p = _to_TYp(m, y)
    dT, dY = _mass_fraction_rhs(m, T, Y, p)
    h = 1e-30
    dC = np.imag(_conc(m, T + 1j * h * dT, Y + 1j * h * dY, p)) / h
    S = oracle.source_terms(m, y, energy=CONST_P_REACTOR)
    scale = oracle.source_sum_scale(m, y, energy=CONST_P_REACTOR)
    np.testing.assert_array_equal(S[:, 0], oracle.source_terms(m, y, energy=CONST_P)[:, 0])
    err = np.abs(S[:, 1:] - dC) / (np.abs(dC) + scale[:, 1:])
    assert err.max() < 1e-12


@pytest.mark.parametrize("name", MECHS)
def test_pressure_and_mass_enthalpy_are_constant(name):
    m = _mech(name)
    y = _states(m, 24, seed=32)
    T, C = y[:, 0], y[:, 1:]
    S = oracle.source_terms(m, y, energy=CONST_P_REACTOR)
    mag = oracle.source_sum_scale(m, y, energy=CONST_P_REACTOR)
    # d(T sum C)/dt = T sum S_i + (sum C) S_T
    dp = T * S[:, 1:].sum(axis=1) + C.sum(axis=1) * S[:, 0]
    assert np.all(np.abs(dp) <= 1e-12 * (T * mag[:, 1:].sum(axis=1) + C.sum(axis=1) * mag[:, 0]))
    # d(sum C_i H_i / rho)/dt = 0 with rho = sum W_i C_i:
    # rho (sum S_i H_i + S_T sum C_i Cp_i) - (sum C_i H_i)(sum W_i S_i) = 0
    cp_R, h_RT = oracle.nasa7_molar(m, T)[:2]
    H, Cp = h_RT * (R * T)[:, None], cp_R * R
    rho = C @ m.W
    d = rho * ((S[:, 1:] * H).sum(axis=1) + S[:, 0] * (C * Cp).sum(axis=1)) - (C * H).sum(axis=1) * (S[:, 1:] @ m.W)
    bound = rho * ((mag[:, 1:] * np.abs(H)).sum(axis=1) + mag[:, 0] * (C * Cp).sum(axis=1)) \
        + np.abs((C * H).sum(axis=1)) * (mag[:, 1:] @ m.W)
    assert np.all(np.abs(d) <= 1e-12 * bound)


def test_thermoneutral_mole_conserving_reaction_reduces_to_constant_pressure():
    from test_oracle_integrators import _isomer_mech
    m = _isomer_mech()
    rng = np.random.default_rng(3)
    y = np.column_stack([rng.uniform(1100.0, 2000.0, 10), rng.uniform(1e-3, 1e-2, (10, 3))])
    S0 = oracle.source_terms(m, y, energy=CONST_P)
    np.testing.assert_allclose(np.abs(S0[:, 0]), 0.0, atol=1e-9 * np.abs(S0[:, 1:]).max())
    np.testing.assert_allclose(oracle.source_terms(m, y, energy=CONST_P_REACTOR), S0, rtol=1e-12,
                               atol=1e-12 * np.abs(S0).max())
    J0 = oracle.jacobian(m, y, energy=CONST_P)
    J2 = oracle.jacobian(m, y, energy=CONST_P_REACTOR)
    # g = 0 here, but dg/dy is not: the difference is -C_i dg/dy_k, nothing else
    c, Om = y[:, 1:].sum(axis=1), S0[:, 1:].sum(axis=1)
    dg = J0[:, 1:, :].sum(axis=1) / c[:, None] + J0[:, 0, :] / y[:, :1]
    dg[:, 1:] -= (Om / c ** 2)[:, None]
    dg[:, 0] -= S0[:, 0] / y[:, 0] ** 2
    np.testing.assert_allclose(J2[:, 1:, :] - J0[:, 1:, :], -y[:, 1:, None] * dg[:, None, :], rtol=1e-9,
                               atol=1e-12 * np.abs(J0).max())


@pytest.mark.parametrize("name", MECHS + ["ch4like_53_325"])
def test_jacobian_matches_complex_step(name):
    m = _mech(name)
    y = _states(m, 10 if m.ns > 20 else 30, seed=33)
    J, M = oracle.jacobian(m, y, energy=CONST_P_REACTOR, magnitude=True)
    Jc = oracle.jacobian_complex_step(m, y, energy=CONST_P_REACTOR)
    assert np.all(M >= np.abs(J) * (1 - 1e-12))
    assert np.all(np.abs(J - Jc) <= 1e-13 * M)
    rel = np.linalg.norm(J - Jc, axis=(1, 2)) / np.linalg.norm(Jc, axis=(1, 2))
    assert rel.max() < 1e-13


def test_dsource_dlnA_matches_complex_step(mech_tiny):
    m = mech_tiny
    y = _states(m, 8, seed=34)
    D = oracle.dsource_dlnA(m, y, energy=CONST_P_REACTOR)
    h = 1e-40
    for j in range(m.nr):
        lnA = m.lnA_default.astype(complex)
        lnA[j] += 1j * h
        col = np.imag(oracle.source_terms(m, y.astype(complex), lnA, CONST_P_REACTOR)) / h
        np.testing.assert_allclose(D[:, :, j], col, rtol=1e-12, atol=1e-12 * np.abs(col).max())


def _radau_reference(m, y0, t_end):
    """Independent stiff solution of the mass-fraction ODE (scipy Radau, tight tolerances)."""
    out = []
    for c in range(y0.shape[0]):
        T0, Y0, p0 = _to_TYp(m, y0[c:c + 1])

        def rhs(_t, u):
            dT, dY = _mass_fraction_rhs(m, u[:1], u[None, 1:], p0)
            return np.concatenate([dT, dY[0]])

        sol = solve_ivp(rhs, (0.0, t_end), np.concatenate([T0, Y0[0]]), method="Radau", rtol=1e-12,
                        atol=np.concatenate([[1e-9], np.full(m.ns, 1e-16)]))
        assert sol.success
        u = sol.y[:, -1]
        C = _conc(m, u[:1], u[None, 1:], p0)[0]
        out.append(np.concatenate([u[:1], C]))
    return np.array(out)


def _rel_err(m, got, ref):
    T, Y, _ = _to_TYp(m, got)
    Tr, Yr, _ = _to_TYp(m, ref)
    return max(np.abs(T - Tr).max() / Tr.max(), np.abs(Y - Yr).max())


def test_integrators_converge_to_the_mass_fraction_ode(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 3)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    t_end = 2e-7
    ref = _radau_reference(m, y0, t_end)
    opt = IntegratorOptions(energy=CONST_P_REACTOR, newton_rtol=1e-12, newton_atol_Y=1e-18, newton_atol_T=1e-10)
    errs = []
    for N in (20, 40, 80):
        r = oracle.integrate_be(m, y0, t_end, N, opt=opt)
        assert np.all(r["status"] == oracle.CELL_OK)
        errs.append(_rel_err(m, r["y"], ref))
    # first order: each halving of the step halves the error
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3
    ro = oracle.integrate_ros2(m, y0, t_end, opt=IntegratorOptions(energy=CONST_P_REACTOR, atol=1e-12))
    assert np.all(ro["status"] == oracle.CELL_OK)
    assert _rel_err(m, ro["y"], ref) < 1e-6
    # the state keeps its pressure and its mass-specific enthalpy to the scheme's accuracy, and the
    # density-holding form does not (it keeps rho instead)
    p0 = R * y0[:, 0] * y0[:, 1:].sum(axis=1)
    p_ro = R * ro["y"][:, 0] * ro["y"][:, 1:].sum(axis=1)
    assert np.abs(p_ro / p0 - 1.0).max() < 1e-7
    held = oracle.integrate_ros2(m, y0, t_end, opt=IntegratorOptions(energy=CONST_P, atol=1e-12))
    p_held = R * held["y"][:, 0] * held["y"][:, 1:].sum(axis=1)
    assert np.abs(p_held / p0 - 1.0).max() > 1e-3


def test_temperature_from_enthalpy_as_constant_pressure(mech_small):
    m = mech_small
    y = _states(m, 16, seed=35)
    e, _ = oracle.energy_density(m, y[:, 1:], y[:, 0], CONST_P)
    T0 = y[:, 0] * 0.9
    np.testing.assert_array_equal(oracle.T_from_energy(m, y[:, 1:], e, T0, CONST_P_REACTOR),
                                  oracle.T_from_energy(m, y[:, 1:], e, T0, CONST_P))


def test_backward_euler_sensitivities_in_reactor_mode(mech_tiny):
    """The backward-Euler tangent in the reactor mode against central differences of the forward
    map in ln A (three reactions), and the adjoint against the tangent (dot-product identity)."""
    from oracle.sensitivity import be_adjoint, be_tangent, final_loss
    from synth.states import loss_weights
    m = mech_tiny
    T, p, Y = sample_config("be_small", m.ns, 3)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    opt = IntegratorOptions(energy=CONST_P_REACTOR)
    fwd = lambda lnA: oracle.integrate_be(m, y0, 1e-7, 12, lnA=lnA, opt=opt, record=True)  # noqa: E731
    r = fwd(None)
    assert np.all(r["status"] == 0)
    s = be_tangent(m, y0, r["trajectory"], energy=CONST_P_REACTOR)
    h = 1e-6
    for j in (0, m.nr // 2, m.nr - 1):
        lp, lm = m.lnA_default.copy(), m.lnA_default.copy()
        lp[j] += h
        lm[j] -= h
        fd = (fwd(lp)["y"] - fwd(lm)["y"]) / (2 * h)
        scale = np.abs(s[:, :, j]).max(axis=1, keepdims=True)
        noise = 1e-15 * np.abs(r["y"]) / h
        assert np.all(np.abs(fd - s[:, :, j]) <= 1e-5 * scale + noise), j
    _, lam = final_loss(m, r["y"], loss_weights(3, m.ns))
    lam0, g = be_adjoint(m, lam, r["trajectory"], energy=CONST_P_REACTOR)
    via_tangent = np.einsum("ci,cik->ck", lam, s)
    np.testing.assert_allclose(g, via_tangent[:, :m.nr], rtol=1e-9, atol=1e-12 * np.abs(g).max())
    np.testing.assert_allclose(lam0, via_tangent[:, m.nr:], rtol=1e-9, atol=1e-12 * np.abs(lam0).max())
