"""Pins of the oracle's GMRES (Section 3.4) and YASS (Appendix A.4) against independent facts.

GMRES (oracle.linsolve.gmres):
* run to the full space it returns LAPACK's solution (numpy.linalg.solve) to rounding;
* its j-th iterate minimises the preconditioned residual over the Krylov space K_j: checked against
  a brute-force least-squares fit over the explicitly formed basis [c, Bc, ..., B^(j-1) c];
* Jacobi preconditioning solves a diagonal system in one iteration; without it a diagonal system
  with k distinct entries needs exactly k (the degree of the minimal polynomial); Gauss-Seidel
  solves a lower-triangular one in one iteration, and its iterates minimise the residual over the
  Krylov space of M^-1 A (brute force);
* GMRES(1) is the minimal-residual iteration x <- x + (r.Br / Br.Br) r;
each with both least-squares solves of the Hessenberg problem (LAPACK lstsq and Givens rotations).

YASS (oracle.integrate_yass):
* on the linear isomerisation A <=> B (T constant) one accepted substep is (I - hK)^-1 C exactly,
  so without halving N steps equal (I - hK)^-N C0, with the LU and with the GMRES solve;
* with a decrement bound that forces halving, the result equals the halving rule carried out with
  those closed-form matrices;
* the h_min failure after the predicted number of halvings, the attempt budget, linear
  invariants, and first order on a mechanism.
"""

import numpy as np
import pytest

import oracle
from oracle.integrate import IntegratorOptions
from oracle.linsolve import gmres
from synth.states import sample_config

from test_oracle_integrators import _isomer_mech, _linear_K, _onto_manifold


def _random_system(n, seed, cond_shift=4.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + cond_shift * np.eye(n)
    return A, rng.standard_normal(n)


LSQ = ["lstsq", "givens"]


@pytest.mark.parametrize("lsq", LSQ)
@pytest.mark.parametrize("jacobi", [True, False])
def test_gmres_full_space_equals_lapack(jacobi, lsq):
    for seed in range(5):
        A, b = _random_system(8, seed)
        x, its, conv = gmres(A, b, 0, 1e-15, 50, jacobi, lsq)
        assert conv and its <= 2 * 8       # n, and at most one short restart at the rounding floor
        ref = np.linalg.solve(A, b)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("lsq", LSQ)
def test_gmres_on_chemistry_iteration_matrix(mech_small, lsq):
    """I - hJ of a synthetic mechanism (badly scaled: T next to concentrations)."""
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 3)
    y = oracle.state_from_TPY(m, T, p, Y)
    J = oracle.jacobian(m, y)
    S = oracle.source_terms(m, y)
    for c in range(3):
        h = 1e-7
        A = np.eye(m.n) - h * J[c]
        b = h * S[c]
        x, its, conv = gmres(A, b, 0, 1e-15, 100, True, lsq)
        ref = np.linalg.solve(A, b)
        assert conv
        assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("lsq", LSQ)
@pytest.mark.parametrize("jacobi", [True, False])
def test_gmres_iterates_minimise_the_residual_over_krylov_space(jacobi, lsq):
    A, b = _random_system(8, 11, cond_shift=3.0)
    dinv = 1.0 / np.diag(A) if jacobi else np.ones(8)
    B, c = dinv[:, None] * A, dinv * b
    for j in range(1, 5):
        x, its, _ = gmres(A, b, 0, 0.0, j, jacobi, lsq)
        assert its == j
        K = np.stack([np.linalg.matrix_power(B, i) @ c for i in range(j)], axis=1)
        z = np.linalg.lstsq(B @ K, c, rcond=None)[0]
        x_ref = K @ z
        assert np.linalg.norm(c - B @ x) == pytest.approx(np.linalg.norm(c - B @ x_ref), rel=1e-10)
        assert np.abs(x - x_ref).max() <= 1e-9 * np.abs(x_ref).max()


@pytest.mark.parametrize("lsq", LSQ)
def test_gmres_diagonal_systems(lsq):
    d = np.array([2.0, 2.0, 5.0, 5.0, 5.0, -3.0, 2.0])
    A = np.diag(d)
    b = np.arange(1.0, 8.0)
    x, its, conv = gmres(A, b, 0, 1e-14, 50, True, lsq)
    assert conv and its == 1
    np.testing.assert_allclose(x, b / d, rtol=1e-15)
    x, its, conv = gmres(A, b, 0, 1e-14, 50, False, lsq)
    assert conv and its == 3
    np.testing.assert_allclose(x, b / d, rtol=1e-13)


@pytest.mark.parametrize("lsq", LSQ)
def test_gmres_gauss_seidel(lsq):
    """M = lower(A): a lower-triangular system is solved in one iteration (M^-1 A = I); in general
    the iterates minimise |M^-1 (b - A x)| over the Krylov space of M^-1 A (brute force with M^-1
    formed by scipy's triangular solve); the full space gives LAPACK's solution."""
    from scipy.linalg import solve_triangular
    A, b = _random_system(7, 21, cond_shift=4.0)
    Lo = np.tril(A)
    x, its, conv = gmres(Lo, b, 0, 1e-14, 20, oracle.linsolve.PRECOND_GS, lsq)
    assert conv and its == 1
    np.testing.assert_allclose(x, np.linalg.solve(Lo, b), rtol=1e-12)
    Minv_A = solve_triangular(Lo, A, lower=True)
    c = solve_triangular(Lo, b, lower=True)
    for j in range(1, 4):
        x, its, _ = gmres(A, b, 0, 0.0, j, oracle.linsolve.PRECOND_GS, lsq)
        K = np.stack([np.linalg.matrix_power(Minv_A, i) @ c for i in range(j)], axis=1)
        x_ref = K @ np.linalg.lstsq(Minv_A @ K, c, rcond=None)[0]
        assert np.abs(x - x_ref).max() <= 1e-9 * np.abs(x_ref).max()
    x, its, conv = gmres(A, b, 0, 1e-15, 30, oracle.linsolve.PRECOND_GS, lsq)
    ref = np.linalg.solve(A, b)
    assert conv and np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("lsq", LSQ)
def test_gmres_restart_one_is_minimal_residual_iteration(lsq):
    A, b = _random_system(6, 3, cond_shift=6.0)
    x_ref = np.zeros(6)
    for _ in range(2):
        r = b - A @ x_ref
        Ar = A @ r
        x_ref = x_ref + (r @ Ar) / (Ar @ Ar) * r
    x, its, _ = gmres(A, b, 1, 0.0, 2, False, lsq)
    assert its == 2
    np.testing.assert_allclose(x, x_ref, rtol=1e-12)


# ----------------------------------------------------------------------------- YASS

def _isomer_setup():
    m = _isomer_mech()
    T = 1400.0
    y0 = np.array([[T, 0.006, 0.001, 0.002]])
    return m, T, y0, _linear_K(m, T)


@pytest.mark.parametrize("solver", [oracle.LINSOLVE_LU, oracle.LINSOLVE_GMRES])
def test_yass_linear_isomerisation_no_halving(solver):
    m, T, y0, K = _isomer_setup()
    tend = 0.5 / abs(K[0, 0])
    for N in (1, 4, 16):
        h = tend / N
        opt = IntegratorOptions(yass_alpha=1e300, linear_solver=solver, krylov_rtol=1e-15)
        r = oracle.integrate_yass(m, y0, tend, N, opt=opt)
        assert r["status"][0] == 0 and r["accepted"][0] == N and r["rejected"][0] == 0
        ref = np.linalg.matrix_power(np.linalg.inv(np.eye(3) - h * K), N) @ y0[0, 1:]
        np.testing.assert_allclose(r["y"][0, 1:], ref, rtol=1e-12, atol=1e-18)
        assert r["y"][0, 0] == T


def _closed_form_halving(C0, K, W, h0, n_steps, alpha):
    """The halving rule with the closed-form substep C <- (I - hK)^-1 C of the linear problem."""
    rho = C0 @ W
    C = C0.copy()
    acc = rej = 0
    for _ in range(n_steps):
        depth, done = 0, 0
        while done < 2 ** depth:
            h = h0 / 2 ** depth
            dC = np.linalg.solve(np.eye(len(C)) - h * K, C) - C
            if np.max(np.abs(dC) * W / rho) <= alpha:
                C = C + dC
                acc += 1
                done += 1
            else:
                rej += 1
                depth += 1
                done *= 2
    return C, acc, rej


def test_yass_linear_isomerisation_with_halving():
    m, T, y0, K = _isomer_setup()
    tend = 3.0 / abs(K[0, 0])
    alpha = 0.02
    C, acc, rej = _closed_form_halving(y0[0, 1:], K, m.W, tend / 2, 2, alpha)
    assert rej >= 3                     # the bound is active
    for solver in (oracle.LINSOLVE_LU, oracle.LINSOLVE_GMRES):
        opt = IntegratorOptions(yass_alpha=alpha, linear_solver=solver, krylov_rtol=1e-15)
        r = oracle.integrate_yass(m, y0, tend, 2, opt=opt)
        assert r["status"][0] == 0
        assert (r["accepted"][0], r["rejected"][0]) == (acc, rej)
        np.testing.assert_allclose(r["y"][0, 1:], C, rtol=1e-12, atol=1e-18)


def test_yass_h_min_failure_and_budget():
    m, T, y0, K = _isomer_setup()
    h0, h_min = 1e-6, 1e-9
    r = oracle.integrate_yass(m, y0, h0, 1, opt=IntegratorOptions(yass_alpha=1e-300, h_min=h_min))
    # the r-th rejection halves to h0 / 2^r; the first one below h_min fails: 2^-10 h0 < 1e-9
    assert r["status"][0] == oracle.CELL_DT_UNDERFLOW
    assert r["rejected"][0] == 10 and r["accepted"][0] == 0
    np.testing.assert_array_equal(r["y"], y0)
    r = oracle.integrate_yass(m, y0, h0, 1, opt=IntegratorOptions(yass_alpha=1e-300, h_min=0.0, max_steps=3))
    assert r["status"][0] == oracle.CELL_MAX_STEPS and r["rejected"][0] == 3


def test_yass_invariants_and_first_order(mech_small):
    m = mech_small
    T, p, Y = sample_config("be_small", m.ns, 6)
    y0 = oracle.state_from_TPY(m, T, p, Y)
    r = oracle.integrate_yass(m, y0, 2e-6, 4)
    assert np.all(r["status"] == 0) and r["rejected"].sum() > 0
    np.testing.assert_allclose(r["y"][:, 1:] @ m.E.T, y0[:, 1:] @ m.E.T, rtol=1e-11)
    np.testing.assert_allclose(r["y"][:, 1:] @ m.W, y0[:, 1:] @ m.W, rtol=1e-12)
    inert = 1 + np.nonzero(m.inert)[0]
    np.testing.assert_allclose(r["y"][:, inert], y0[:, inert], rtol=1e-13)
    # first order (no halving at these steps) against a fine Rosenbrock reference
    y1 = _onto_manifold(m)
    t = 2e-9
    ref = oracle.integrate_ros2(m, y1, t, fixed_steps=512)["y"]
    e = []
    for N in (16, 32, 64, 128):
        rr = oracle.integrate_yass(m, y1, t, N, opt=IntegratorOptions(yass_alpha=1e300))
        e.append(np.abs(rr["y"][:, 1:] - ref[:, 1:]).max())
    o = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.median(o) == pytest.approx(1.0, abs=0.25), o
