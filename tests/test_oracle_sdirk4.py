"""Pins of the oracle's SDIRK-4 (Appendix A.2: five stages, the printed 7-digit tableau, a_52 read
as b_2).

* the tableau satisfies the eight order conditions of order 4 (sum b = 1, b.c = 1/2, b.c^2 = 1/3,
  b.Ac = 1/6, b.c^3 = 1/4, b.(c*Ac) = 1/8, b.A(c^2) = 1/12, b.A^2 c = 1/24) to the 7-digit
  rounding of the printed values (this is what fixes a_52: any other value breaks them by far
  more), and the row sums c_i = sum_j a_ij give c_5 = 1 (stiffly accurate);
* on the linear isomerisation one step is the textbook stability function
  R(z) = 1 + z b^T (I - zA)^-1 1 applied to hK (through the eigen-decomposition of K), to
  rounding, and R(z) -> 1 - b^T A^-1 1 = 0 for z -> -inf;
* order 4 against expm on the linear problem and on a synthetic mechanism, at step sizes where
  the truncation error stays above the ~1e-7 defects of the 7-digit coefficients.
"""

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle.integrate import SDIRK4_A, SDIRK4_B, IntegratorOptions

from test_oracle_integrators import _isomer_mech, _linear_K, _onto_manifold

A, B = SDIRK4_A, SDIRK4_B
C = A.sum(axis=1)


def test_order_conditions():
    Ac = A @ C
    conds = [B.sum() - 1, B @ C - 1 / 2, B @ C**2 - 1 / 3, B @ Ac - 1 / 6, B @ C**3 - 1 / 4,
             B @ (C * Ac) - 1 / 8, B @ (A @ C**2) - 1 / 12, B @ (A @ Ac) - 1 / 24]
    assert np.max(np.abs(conds)) < 1e-6, conds
    assert C[-1] == pytest.approx(1.0, abs=1e-6)
    # a_52 is what makes them hold: a different value breaks the order-2 condition at once
    A2 = A.copy()
    A2[4, 1] = 0.0
    assert abs(B @ A2.sum(axis=1) - 0.5) > 0.1 or abs(A2.sum(axis=1)[-1] - 1.0) > 0.1


def _R(z):
    n = len(B)
    return 1.0 + z * (B @ np.linalg.solve(np.eye(n) - z * A, np.ones(n)))


def test_linear_isomerisation_stability_function_and_order():
    m = _isomer_mech()
    T = 1400.0
    y0 = np.array([[T, 0.006, 0.001, 0.002]])
    K = _linear_K(m, T)
    w, V = np.linalg.eig(K)
    # hK from 2 to 0.25: errors 3e-5 .. 5e-9, above the ~5e-10 floor of the 7-digit coefficients
    tend = 2.0 / abs(K[0, 0])
    exact = expm(K * tend) @ y0[0, 1:]
    errs = []
    for N in (1, 2, 4, 8):
        h = tend / N
        r = oracle.integrate_sdirk4(m, y0, tend, N)
        assert r["status"][0] == 0
        Rh = (V @ np.diag([_R(h * lam) for lam in w]) @ np.linalg.inv(V)).real
        ref = np.linalg.matrix_power(Rh, N) @ y0[0, 1:]
        np.testing.assert_allclose(r["y"][0, 1:], ref, rtol=1e-11, atol=1e-18)
        errs.append(np.abs(r["y"][0, 1:] - exact).max())
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.median(o) == pytest.approx(4.0, abs=0.35), o
    assert abs(_R(-1e9)) < 1e-5


def test_convergence_order_on_mechanism(mech_small):
    """Refinement against the scheme's own solution at 128 steps, with a Newton tolerance far below
    the truncation errors (4e-10 .. 2e-12 here)."""
    m = mech_small
    y0 = _onto_manifold(m)
    t = 1e-7
    tight = IntegratorOptions(newton_rtol=1e-15, newton_atol_T=1e-13, newton_atol_Y=1e-20)
    ref = oracle.integrate_sdirk4(m, y0, t, 128, opt=tight)["y"]
    e = []
    for N in (2, 4, 8):
        r = oracle.integrate_sdirk4(m, y0, t, N, opt=tight)
        assert np.all(r["status"] == 0)
        e.append(np.abs(r["y"][:, 1:] - ref[:, 1:]).max())
    o = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.median(o) == pytest.approx(4.0, abs=0.3), (e, o)
