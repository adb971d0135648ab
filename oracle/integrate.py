"""Per-cell implicit integration over one operator-split step (paper Section 3 and Appendix A).

* ``state_from_TPY`` / ``mass_fractions``: the map (T, p, Y) -> y = (T, C) with
  rho = p Wbar / (R T), C_i = rho Y_i / W_i, and back Y_i = W_i C_i / rho (Section 2).
* ``integrate_be``: backward Euler, y^{n+1} - y^n = dt S(y^{n+1}), solved by full Newton
  (eqs. Backward_euler, newtons-method-2, jacobian: G = I/dt - J re-evaluated every
  iteration).  A step whose Newton iteration fails is split into two halves, recursively,
  as YASS halves its step (Appendix A.4), down to a maximum depth.
* ``integrate_sdirk2`` / ``integrate_sdirk4``: the two-stage SDIRK scheme of Appendix A.1
  (gamma = 1 - sqrt(2)/2) and the five-stage one of Appendix A.2 at fixed steps, each stage
  solved by full Newton from the initial guess S(y_n).
* ``integrate_yass``: YASS (Appendix A.4): one linearised backward-Euler solve
  (I - h J(y_n)) dy = h S(y_n) per substep, the substep halved while the decrement is larger
  than alpha, failure once it would fall below h_min; the solve by LU or by GMRES with Jacobi,
  Gauss-Seidel or no preconditioning (Section 3.4, ``oracle.linsolve``).
* ``integrate_ros2``: the two-stage Rosenbrock method of Appendix A.3 with
  gamma = 1 + sqrt(2)/2, alpha = 1/gamma, beta = -2/gamma, m1 = 3/(2 gamma),
  m2 = 1/(2 gamma); the second stage right-hand side is S(y + alpha G1) + (beta/h) G1
  (the printed extra "- S(y_n)" term is read as a typesetting slip: with it the scheme is
  not consistent).  The paper runs it at fixed steps; here it also carries an embedded
  first-order solution y + G1/gamma, a weighted RMS error norm and a step-size
  controller so that one call covers a whole split step.

Linear solves use LAPACK (numpy.linalg.solve: LU with partial pivoting).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .kinetics import CONST_P, jacobian, source_terms
from .linsolve import gmres
from .mechanism import R

CELL_OK, CELL_NEWTON_FAIL, CELL_DT_UNDERFLOW, CELL_MAX_STEPS, CELL_NONFINITE, CELL_T_RANGE = range(6)
LINSOLVE_LU, LINSOLVE_GMRES = 0, 1

ROS2_GAMMA = 1.0 + math.sqrt(2.0) / 2.0
ROS2_ALPHA = 1.0 / ROS2_GAMMA
ROS2_BETA = -2.0 / ROS2_GAMMA
ROS2_M1 = 3.0 / (2.0 * ROS2_GAMMA)
ROS2_M2 = 1.0 / (2.0 * ROS2_GAMMA)


@dataclass
class IntegratorOptions:
    energy: int = CONST_P
    # backward Euler / Newton
    newton_max: int = 10
    newton_rtol: float = 1e-10      # on T and on mass fractions
    newton_atol_T: float = 1e-8     # K
    newton_atol_Y: float = 1e-14    # mass fraction
    halving_max_depth: int = 8
    # Rosenbrock controller
    rtol: float = 1e-6
    atol: float = 1e-10             # on mass fractions, and in K on T
    h_min: float = 1e-20
    max_steps: int = 100000
    fac_min: float = 0.2
    fac_max: float = 5.0
    safety: float = 0.9
    # YASS (Appendix A.4) and its linear solver (Section 3.4)
    yass_alpha: float = 0.1         # bound on max(|dT|/T, max_i |dY_i|) per substep
    linear_solver: int = 0          # LINSOLVE_LU or LINSOLVE_GMRES
    krylov_dim: int = 0             # GMRES restart length (0: the system size)
    krylov_rtol: float = 1e-12      # on the preconditioned residual, relative to |M^-1 b|
    krylov_max_iter: int = 100
    krylov_precond: int = 1         # 0: M = I, 1: Jacobi M = diag(A), 2: Gauss-Seidel M = lower(A)
    krylov_lsq: str = "lstsq"       # GMRES least-squares solve: "lstsq" or "givens"


def state_from_TPY(mech, T, p, Y):
    """(T, p, Y) -> y = (T, C): rho = p Wbar/(R T), Wbar = 1/sum(Y/W), C = rho Y / W."""
    T = np.asarray(T, dtype=float)
    Y = np.asarray(Y, dtype=float)
    Wbar = 1.0 / (Y / mech.W[None, :]).sum(axis=1)
    rho = np.asarray(p) * Wbar / (R * T)
    C = rho[:, None] * Y / mech.W[None, :]
    return np.concatenate([T[:, None], C], axis=1)


def mass_fractions(mech, y):
    """Y_i = W_i C_i / sum_k W_k C_k."""
    C = np.asarray(y)[:, 1:]
    rhoY = C * mech.W[None, :]
    return rhoY / rhoY.sum(axis=1, keepdims=True)


def _input_status(y):
    st = np.zeros(y.shape[0], dtype=np.int32)
    st[~np.all(np.isfinite(y), axis=1)] = CELL_NONFINITE
    st[(st == CELL_OK) & ~(y[:, 0] > 0.0)] = CELL_T_RANGE
    return st


# ----------------------------------------------------------------------------- backward Euler

def _newton_scale(mech, y, rho, opt):
    """Per-component Newton scale: T: rtol T + atol_T; C_i: (atol_Y + rtol |Y_i|) rho / W_i."""
    sc = np.empty_like(y)
    sc[:, 0] = opt.newton_rtol * np.abs(y[:, 0]) + opt.newton_atol_T
    Y = np.abs(y[:, 1:]) * mech.W[None, :] / rho[:, None]
    sc[:, 1:] = (opt.newton_atol_Y + opt.newton_rtol * Y) * rho[:, None] / mech.W[None, :]
    return sc


def be_newton(mech, y_n, dt, lnA, opt, rho=None):
    """Solve y - y_n - dt S(y) = 0 for every cell of y_n (shape [m, n]) by full Newton.

    Returns (y, converged[m], iterations[m]).  Iteration k solves
    (I/dt - J(y_k)) delta = -((y_k - y_n)/dt - S(y_k)) and sets y_{k+1} = y_k + delta.  It
    has converged when max_i |delta_i| / sc_i <= 1 (scales from y_{k+1}); it has failed
    when the scaled norm grows from iteration 2 on, when y_{k+1} is not finite or has
    T <= 0, or when ``newton_max`` iterations pass without convergence.

    ``rho`` [m]: the density in the scales, by default that of y_n.  The integrators pass the
    density of the state at the start of the integration: it is a constant of the motion in the
    density-holding energy modes, and in the reactor mode (whose density changes) it keeps the
    scales fixed over the call.
    """
    m, n = y_n.shape
    if rho is None:
        rho = (y_n[:, 1:] * mech.W[None, :]).sum(axis=1)
    y = y_n.copy()
    active = np.ones(m, dtype=bool)
    conv = np.zeros(m, dtype=bool)
    iters = np.zeros(m, dtype=np.int32)
    prev = np.full(m, np.inf)
    eye = np.eye(n)
    for k in range(opt.newton_max):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        yk = y[idx]
        f = (yk - y_n[idx]) / dt - source_terms(mech, yk, lnA, opt.energy)
        G = eye[None] / dt - jacobian(mech, yk, lnA, opt.energy)
        with np.errstate(all="ignore"):
            try:
                delta = np.linalg.solve(G, -f[:, :, None])[:, :, 0]
            except np.linalg.LinAlgError:
                delta = np.full_like(yk, np.nan)
                for c in range(idx.size):
                    try:
                        delta[c] = np.linalg.solve(G[c], -f[c])
                    except np.linalg.LinAlgError:
                        pass
            ynew = yk + delta
            norm = np.max(np.abs(delta) / _newton_scale(mech, ynew, rho[idx], opt), axis=1)
        iters[idx] += 1
        bad = ~np.all(np.isfinite(ynew), axis=1) | ~(ynew[:, 0] > 0.0) | ~np.isfinite(norm)
        diverged = (k >= 2) & (norm > prev[idx])
        done = ~bad & (norm <= 1.0)
        y[idx] = np.where(bad[:, None], yk, ynew)
        conv[idx[done]] = True
        stop = bad | done | diverged
        active[idx[stop]] = False
        prev[idx] = norm
    return y, conv, iters


def _be_substep_recursive(mech, y, dt, lnA, opt, depth, record, rho):
    """One step of size dt for a single cell, halving on Newton failure (depth-first)."""
    ynew, conv, it = be_newton(mech, y[None], dt, lnA, opt, np.array([rho]))
    newton = int(it[0])
    if conv[0]:
        if record is not None:
            record.append((ynew[0].copy(), dt))
        return ynew[0], True, newton
    if depth >= opt.halving_max_depth:
        return y, False, newton
    ymid, ok, n1 = _be_substep_recursive(mech, y, 0.5 * dt, lnA, opt, depth + 1, record, rho)
    newton += n1
    if not ok:
        return ymid, False, newton
    yend, ok, n2 = _be_substep_recursive(mech, ymid, 0.5 * dt, lnA, opt, depth + 1, record, rho)
    return yend, ok, newton + n2


def integrate_be(mech, y0, dt_total, n_steps, lnA=None, opt=None, record=False):
    """Backward Euler over ``n_steps`` fixed steps of dt_total/n_steps for every cell.

    Returns dict(y, status, steps, newton, [trajectory]).  ``steps`` counts completed full
    steps per cell (a cell-substep each); ``newton`` counts Newton iterations.  With
    ``record`` the per-cell list of (y_end, dt_sub) of every accepted (sub)step is returned.
    """
    opt = opt or IntegratorOptions()
    y = np.array(y0, dtype=float, copy=True)
    nc = y.shape[0]
    status = _input_status(y)
    steps = np.zeros(nc, dtype=np.int32)
    newton = np.zeros(nc, dtype=np.int64)
    traj = [[] for _ in range(nc)] if record else None
    dt = dt_total / n_steps
    rho0 = (y[:, 1:] * mech.W[None, :]).sum(axis=1)
    for _ in range(n_steps):
        idx = np.nonzero(status == CELL_OK)[0]
        if idx.size == 0:
            break
        ynew, conv, it = be_newton(mech, y[idx], dt, lnA, opt, rho0[idx])
        newton[idx] += it
        for c, ok, yc in zip(idx, conv, ynew):
            if ok:
                y[c] = yc
                steps[c] += 1
                if record:
                    traj[c].append((yc.copy(), dt))
        for c in idx[~conv]:
            if opt.halving_max_depth < 1:
                status[c] = CELL_NEWTON_FAIL
                continue
            # the whole step failed: split it into two halves, recursively
            rec = [] if record else None
            y1, ok, n1 = _be_substep_recursive(mech, y[c], 0.5 * dt, lnA, opt, 1, rec, rho0[c])
            newton[c] += n1
            if ok:
                y2, ok, n2 = _be_substep_recursive(mech, y1, 0.5 * dt, lnA, opt, 1, rec, rho0[c])
                newton[c] += n2
                y1 = y2
            y[c] = y1
            if record:
                traj[c].extend(rec)
            if ok:
                steps[c] += 1
            else:
                status[c] = CELL_NEWTON_FAIL
    out = dict(y=y, status=status, steps=steps, newton=newton)
    if record:
        out["trajectory"] = traj
    return out


# ----------------------------------------------------------------------------- SDIRK-2

SDIRK2_GAMMA = 1.0 - math.sqrt(2.0) / 2.0


def _sdirk_stage(mech, base, gh, guess, rho, lnA, opt):
    """Newton for one SDIRK stage of every cell: Gamma = S(base + gh Gamma), gh = a_pp h.

    Iteration k solves (I - gamma h J(Y_k)) delta = -(Gamma_k - S(Y_k)) with
    Y_k = base + gamma h Gamma_k and sets Gamma_{k+1} = Gamma_k + delta (Appendix A.1, eqs.
    newtons-method-sdirk2*).  The decrement test reads the state change gamma h delta in the
    backward-Euler Newton scales (scales from Y_{k+1}); failure as for backward Euler: the scaled
    norm grows from iteration 2 on, a non-finite or T <= 0 stage state, or ``newton_max``
    iterations.  Returns (Gamma, converged, iterations).
    """
    m, n = base.shape
    gam = guess.copy()
    active = np.ones(m, dtype=bool)
    conv = np.zeros(m, dtype=bool)
    iters = np.zeros(m, dtype=np.int32)
    prev = np.full(m, np.inf)
    eye = np.eye(n)
    for k in range(opt.newton_max):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        Yk = base[idx] + gh * gam[idx]
        f = gam[idx] - source_terms(mech, Yk, lnA, opt.energy)
        G = eye[None] - gh * jacobian(mech, Yk, lnA, opt.energy)
        with np.errstate(all="ignore"):
            delta = np.full_like(Yk, np.nan)
            for c in range(idx.size):
                try:
                    delta[c] = np.linalg.solve(G[c], -f[c])
                except np.linalg.LinAlgError:
                    pass
            gnew = gam[idx] + delta
            Ynew = base[idx] + gh * gnew
            norm = np.max(np.abs(gh * delta) / _newton_scale(mech, Ynew, rho[idx], opt), axis=1)
        iters[idx] += 1
        bad = ~np.all(np.isfinite(Ynew), axis=1) | ~(Ynew[:, 0] > 0.0) | ~np.isfinite(norm)
        diverged = (k >= 2) & (norm > prev[idx])
        done = ~bad & (norm <= 1.0)
        gam[idx] = np.where(bad[:, None], gam[idx], gnew)
        conv[idx[done]] = True
        stop = bad | done | diverged
        active[idx[stop]] = False
        prev[idx] = norm
    return gam, conv, iters


# Butcher tableaus (A lower triangular with a constant diagonal, weights b).  SDIRK-2: Appendix
# A.1.  SDIRK-4: the five-stage tableau printed in Appendix A.2 (7 significant digits), whose
# a_52 is not printed; it is read as a_52 = b_2, which with a_51 = b_1, a_53 = b_3, a_54 = b_4 and
# a_55 = b_5 as printed makes the scheme stiffly accurate (last row of A = b).
SDIRK2_A = np.array([[SDIRK2_GAMMA, 0.0], [1.0 - SDIRK2_GAMMA, SDIRK2_GAMMA]])
SDIRK2_B = np.array([1.0 - SDIRK2_GAMMA, SDIRK2_GAMMA])
_G4 = 4.0 / 15.0
SDIRK4_B = np.array([2.100115, -7.677800e-1, 2.399816, -2.998818, _G4])
SDIRK4_A = np.array([
    [_G4, 0.0, 0.0, 0.0, 0.0],
    [0.5, _G4, 0.0, 0.0, 0.0],
    [3.541539e-1, -5.415395e-2, _G4, 0.0, 0.0],
    [8.515494e-2, -6.484332e-2, 7.915325e-2, _G4, 0.0],
    [2.100115, -7.677800e-1, 2.399816, -2.998818, _G4],
])


def sdirk_step(mech, y, h, A, b, lnA, opt):
    """One step of the SDIRK scheme (A, b) of size h for every cell of y ([m, n]):

        Gamma_p = S(y + h sum_{j<p} a_pj Gamma_j + a_pp h Gamma_p),  y' = y + h sum_p b_p Gamma_p,

    each stage solved by Newton from the initial guess S(y) (Appendix A.1/A.2).  A cell whose
    stage fails skips the later stages.  Returns (y', converged, iterations)."""
    rho = (y[:, 1:] * mech.W[None, :]).sum(axis=1)
    S0 = source_terms(mech, y, lnA, opt.energy)
    gams = []
    ok = np.ones(y.shape[0], dtype=bool)
    iters = np.zeros(y.shape[0], dtype=np.int32)
    for p in range(len(b)):
        base = y.copy()
        for j in range(p):
            base = base + (h * A[p, j]) * gams[j]
        gp, cp, ip = _sdirk_stage(mech, base, h * A[p, p], S0, rho, lnA, opt)
        iters += np.where(ok, ip, 0)
        ok &= cp
        gams.append(gp)
    ynew = y.copy()
    for p in range(len(b)):
        ynew = ynew + (h * b[p]) * gams[p]
    ok &= np.all(np.isfinite(ynew), axis=1) & (ynew[:, 0] > 0.0)
    return ynew, ok, iters


def sdirk2_step(mech, y, h, lnA, opt):
    """One SDIRK-2 step (Appendix A.1) of size h for every cell of y ([m, n]):

        Gamma1 = S(y + gamma h Gamma1),  Gamma2 = S(y + (1 - gamma) h Gamma1 + gamma h Gamma2),
        y' = y + h ((1 - gamma) Gamma1 + gamma Gamma2),  gamma = 1 - sqrt(2)/2,

    each stage solved by Newton from the initial guess S(y).  Returns (y', converged, iterations).
    """
    return sdirk_step(mech, y, h, SDIRK2_A, SDIRK2_B, lnA, opt)


def integrate_sdirk(mech, y0, dt_total, n_steps, A, b, lnA=None, opt=None):
    """An SDIRK scheme (A, b) over ``n_steps`` fixed steps of dt_total/n_steps for every cell (the
    paper's use, Table 5).  A cell whose step fails keeps its last state and gets
    CELL_NEWTON_FAIL (the paper names no fallback for the SDIRK schemes).  Returns dict(y, status,
    steps, newton)."""
    opt = opt or IntegratorOptions()
    y = np.array(y0, dtype=float, copy=True)
    nc = y.shape[0]
    status = _input_status(y)
    steps = np.zeros(nc, dtype=np.int32)
    newton = np.zeros(nc, dtype=np.int64)
    h = dt_total / n_steps
    for _ in range(n_steps):
        idx = np.nonzero(status == CELL_OK)[0]
        if idx.size == 0:
            break
        ynew, ok, it = sdirk_step(mech, y[idx], h, A, b, lnA, opt)
        newton[idx] += it
        y[idx[ok]] = ynew[ok]
        steps[idx[ok]] += 1
        status[idx[~ok]] = CELL_NEWTON_FAIL
    return dict(y=y, status=status, steps=steps, newton=newton)


def integrate_sdirk2(mech, y0, dt_total, n_steps, lnA=None, opt=None):
    """SDIRK-2 (Appendix A.1) at fixed steps; see ``integrate_sdirk``."""
    return integrate_sdirk(mech, y0, dt_total, n_steps, SDIRK2_A, SDIRK2_B, lnA, opt)


def integrate_sdirk4(mech, y0, dt_total, n_steps, lnA=None, opt=None):
    """SDIRK-4 (Appendix A.2, five stages) at fixed steps; see ``integrate_sdirk``."""
    return integrate_sdirk(mech, y0, dt_total, n_steps, SDIRK4_A, SDIRK4_B, lnA, opt)


# ----------------------------------------------------------------------------- Rosenbrock

def yass_norm(mech, y, dy, rho):
    """Size of a YASS decrement: max(|dT| / T, max_i |dC_i| W_i / rho), the relative change of T
    and the absolute change of the mass fractions (rho from the cell's initial state)."""
    dT = np.abs(dy[:, 0]) / y[:, 0]
    dY = np.abs(dy[:, 1:]) * mech.W[None, :] / rho[:, None]
    return np.maximum(dT, dY.max(axis=1))


def _linear_solve(A, b, opt):
    """One solve of A x = b (single system): LU with partial pivoting (LAPACK) or GMRES.
    Returns (x, Krylov iterations)."""
    if opt.linear_solver == LINSOLVE_GMRES:
        x, its, _ = gmres(A, b, opt.krylov_dim, opt.krylov_rtol, opt.krylov_max_iter, opt.krylov_precond,
                          opt.krylov_lsq)
        return x, its
    return np.linalg.solve(A, b), 0


def integrate_yass(mech, y0, dt_total, n_steps, lnA=None, opt=None):
    """YASS (Appendix A.4) over ``n_steps`` fixed steps of dt_total/n_steps for every cell.

    Each fixed step starts with the substep h = dt_total/n_steps.  An attempt solves
    (I - h J(y)) dy = h S(y) at the current state y (one linearised backward-Euler step).  It is
    accepted when dy, y + dy are finite, T + dT > 0 and yass_norm(dy) <= yass_alpha: then
    y <- y + dy.  Otherwise the substep is halved (h <- h/2) and the attempt repeated; if the halved
    substep is below h_min the cell fails with CELL_DT_UNDERFLOW.  A halved substep is kept until
    the fixed step is covered (the remaining time is always a whole number of substeps); the next
    fixed step starts again from dt_total/n_steps.  A cell that uses up max_steps attempts stops
    with CELL_MAX_STEPS.  A failed cell keeps its last accepted state.
    Returns dict(y, status, accepted, rejected, krylov) (Krylov iterations summed over attempts,
    0 with the LU solver)."""
    opt = opt or IntegratorOptions()
    y = np.array(y0, dtype=float, copy=True)
    nc, n = y.shape
    status = _input_status(y)
    rho = (y[:, 1:] * mech.W[None, :]).sum(axis=1)
    h0 = dt_total / n_steps
    step = np.zeros(nc, dtype=np.int64)
    depth = np.zeros(nc, dtype=np.int64)
    done_sub = np.zeros(nc, dtype=np.int64)      # substeps taken in this fixed step, at this depth
    acc = np.zeros(nc, dtype=np.int64)
    rej = np.zeros(nc, dtype=np.int64)
    kry = np.zeros(nc, dtype=np.int64)
    active = status == CELL_OK
    eye = np.eye(n)
    while active.any():
        idx = np.nonzero(active)[0]
        h = h0 * np.exp2(-depth[idx].astype(float))
        with np.errstate(all="ignore"):
            S = source_terms(mech, y[idx], lnA, opt.energy)
            J = jacobian(mech, y[idx], lnA, opt.energy)
            dy = np.full((idx.size, n), np.nan)
            for c in range(idx.size):
                try:
                    dy[c], its = _linear_solve(eye - h[c] * J[c], h[c] * S[c], opt)
                    kry[idx[c]] += its
                except np.linalg.LinAlgError:
                    pass
            ynew = y[idx] + dy
            norm = yass_norm(mech, y[idx], dy, rho[idx])
        ok = (np.all(np.isfinite(dy), axis=1) & np.all(np.isfinite(ynew), axis=1) & (ynew[:, 0] > 0.0)
              & (norm <= opt.yass_alpha))
        att = acc[idx] + rej[idx] + 1
        for c, cell in enumerate(idx):
            if ok[c]:
                y[cell] = ynew[c]
                acc[cell] += 1
                done_sub[cell] += 1
                if done_sub[cell] == (1 << int(depth[cell])):
                    step[cell] += 1
                    depth[cell] = 0
                    done_sub[cell] = 0
                    if step[cell] == n_steps:
                        active[cell] = False
                        continue
            else:
                rej[cell] += 1
                depth[cell] += 1
                done_sub[cell] *= 2
                if h[c] * 0.5 < opt.h_min or depth[cell] > 60:
                    status[cell] = CELL_DT_UNDERFLOW
                    active[cell] = False
                    continue
            if att[c] >= opt.max_steps:
                status[cell] = CELL_MAX_STEPS
                active[cell] = False
    return dict(y=y, status=status, accepted=acc, rejected=rej, krylov=kry)


def _ros2_scales(mech, y_a, y_b, rho, opt):
    """Error weights: T: rtol max(|T_a|,|T_b|) + atol; species in mass-fraction space."""
    sc = np.empty_like(y_a)
    sc[:, 0] = opt.rtol * np.maximum(np.abs(y_a[:, 0]), np.abs(y_b[:, 0])) + opt.atol
    Ya = np.abs(y_a[:, 1:]) * mech.W[None, :] / rho[:, None]
    Yb = np.abs(y_b[:, 1:]) * mech.W[None, :] / rho[:, None]
    sc[:, 1:] = opt.atol + opt.rtol * np.maximum(Ya, Yb)
    return sc


def _to_mass_space(mech, v, rho):
    """Express a state-shaped vector in (K, mass fraction) units: C components times W_i/rho."""
    out = np.array(v, copy=True)
    out[:, 1:] = v[:, 1:] * mech.W[None, :] / rho[:, None]
    return out


def _wrms(v, sc):
    return np.sqrt(np.mean((v / sc) ** 2, axis=1))


def ros2_initial_step(mech, y, S, dt, rho, opt):
    """h0 = 0.01 ||y|| / ||S(y)|| in the weighted RMS norm, clipped to [h_min, dt]."""
    sc = _ros2_scales(mech, y, y, rho, opt)
    d0 = _wrms(_to_mass_space(mech, y, rho), sc)
    d1 = _wrms(_to_mass_space(mech, S, rho), sc)
    with np.errstate(divide="ignore", invalid="ignore"):
        h0 = np.where(d1 > 0.0, 0.01 * d0 / d1, dt)
    h0 = np.where(np.isfinite(h0), h0, opt.h_min)
    return np.clip(h0, opt.h_min, dt)


def integrate_ros2(mech, y0, dt, lnA=None, opt=None, record=False, fixed_steps=0):
    """Two-stage Rosenbrock from t = 0 to t = dt for every cell (adaptive unless ``fixed_steps``).

    With ``fixed_steps`` > 0 every attempt uses h = dt / fixed_steps and is accepted (the
    paper's fixed-step use, Table 5); otherwise the step is controlled as follows.

    Each attempt with step h:
        G  = I/(gamma h) - J(y_n)
        G Gamma1 = S(y_n)
        G Gamma2 = S(y_n + alpha Gamma1) + (beta / h) Gamma1
        y_{n+1} = y_n + m1 Gamma1 + m2 Gamma2,   e = (Gamma1 + Gamma2) / (2 gamma)
    err = WRMS of e (species converted to mass fractions).  Accept if err <= 1 and the new
    state is finite with T > 0.  New step h * min(fac_max, max(fac_min, 0.9 err^-1/2)),
    growth capped at 1 right after a rejection; the last step is clipped to t_end.
    Returns dict(y, status, accepted, rejected).
    """
    opt = opt or IntegratorOptions()
    y = np.array(y0, dtype=float, copy=True)
    nc, n = y.shape
    status = _input_status(y)
    rho = (y[:, 1:] * mech.W[None, :]).sum(axis=1)
    t = np.zeros(nc)
    h = np.zeros(nc)
    last_rejected = np.zeros(nc, dtype=bool)
    started = np.zeros(nc, dtype=bool)
    accepted = np.zeros(nc, dtype=np.int32)
    rejected = np.zeros(nc, dtype=np.int32)
    active = status == CELL_OK
    eye = np.eye(n)
    hist = [[] for _ in range(nc)] if record else None
    while np.any(active):
        idx = np.nonzero(active)[0]
        yn = y[idx]
        S0 = source_terms(mech, yn, lnA, opt.energy)
        J = jacobian(mech, yn, lnA, opt.energy)
        new = ~started[idx]
        if fixed_steps > 0 and np.any(new):
            h[idx[new]] = dt / fixed_steps
            started[idx[new]] = True
        if np.any(new) and fixed_steps <= 0:
            h[idx[new]] = ros2_initial_step(mech, yn[new], S0[new], dt, rho[idx[new]], opt)
            started[idx[new]] = True
        rem = dt - t[idx]
        last = h[idx] >= rem                      # this attempt reaches the end of the split step
        if fixed_steps > 0:
            last = accepted[idx] + 1 >= fixed_steps
        hh = np.where(last, rem, h[idx])
        with np.errstate(all="ignore"):
            G = eye[None] / (ROS2_GAMMA * hh)[:, None, None] - J
            try:
                G1 = np.linalg.solve(G, S0[:, :, None])[:, :, 0]
            except np.linalg.LinAlgError:
                G1 = np.full_like(yn, np.nan)
            ystar = yn + ROS2_ALPHA * G1
            S1 = source_terms(mech, ystar, lnA, opt.energy)
            rhs = S1 + (ROS2_BETA / hh)[:, None] * G1
            try:
                G2 = np.linalg.solve(G, rhs[:, :, None])[:, :, 0]
            except np.linalg.LinAlgError:
                G2 = np.full_like(yn, np.nan)
            ynew = yn + ROS2_M1 * G1 + ROS2_M2 * G2
            e = (G1 + G2) / (2.0 * ROS2_GAMMA)
            sc = _ros2_scales(mech, yn, ynew, rho[idx], opt)
            err = _wrms(_to_mass_space(mech, e, rho[idx]), sc)
        ok = np.isfinite(err) & np.all(np.isfinite(ynew), axis=1) & (ynew[:, 0] > 0.0)
        acc = ok & ((err <= 1.0) | (fixed_steps > 0))
        with np.errstate(divide="ignore", invalid="ignore"):
            fac = opt.safety / np.sqrt(err)
        fac = np.where(ok, fac, opt.fac_min)
        fac = np.where(np.isnan(fac), opt.fac_max, fac)
        grow_cap = np.where(last_rejected[idx], 1.0, opt.fac_max)
        fac_acc = np.minimum(grow_cap, np.maximum(opt.fac_min, fac))
        fac_rej = np.maximum(opt.fac_min, np.minimum(1.0, fac))
        for c_local, c in enumerate(idx):
            if acc[c_local]:
                y[c] = ynew[c_local]
                t[c] = dt if last[c_local] else t[c] + hh[c_local]
                accepted[c] += 1
                h[c] = hh[c_local] * fac_acc[c_local] if fixed_steps <= 0 else dt / fixed_steps
                last_rejected[c] = False
                if record:
                    hist[c].append((hh[c_local], float(err[c_local])))
                if last[c_local]:
                    active[c] = False
            else:
                rejected[c] += 1
                h[c] = hh[c_local] * fac_rej[c_local]
                last_rejected[c] = True
                if h[c] < opt.h_min:
                    status[c] = CELL_DT_UNDERFLOW
                    active[c] = False
            if active[c] and accepted[c] + rejected[c] >= opt.max_steps:
                status[c] = CELL_MAX_STEPS
                active[c] = False
    out = dict(y=y, status=status, accepted=accepted, rejected=rejected)
    if record:
        out["history"] = hist
    return out
