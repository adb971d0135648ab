"""Forward (tangent) and reverse (discrete adjoint) sensitivities of the integrators.

Each accepted (sub)step of size dt solves F(y', y, theta) = (y' - y)/dt - S(y', theta) = 0.
With A = dF/dy' = I/dt - J(y'):

* tangent:  A s' = s / dt + dS/dtheta(y')                     (s = dy/dtheta)
* adjoint:  A^T mu = lambda',  lambda = mu / dt,  g_theta += mu^T dS/dtheta(y')

theta = (ln A_1..ln A_nr, y0).  The loss of the differentiation workload is
L = sum_cells [T_N + sum_i w_i Y_i(y_N)] with Y_i = W_i C_i / sum_k W_k C_k, and the
initial state comes from (T0, p, Y0) through rho0 = p Wbar/(R T0), C_i = rho0 Y_i / W_i.

The two-stage Rosenbrock scheme (Appendix A.3) is differentiated along its accepted step
sequence, held fixed (the step-size controller is not differentiated).  One step of size h from y:

    G = I/(gamma h) - J(y),  G g1 = S(y),  y* = y + alpha g1,  G g2 = S(y*) + (beta/h) g1,
    y' = y + m1 g1 + m2 g2.

Its adjoint, from the stationarity of the step's Lagrangian, with lambda = dL/dy':

    G^T u2 = m2 lambda
    G^T u1 = m1 lambda + alpha J(y*)^T u2 + (beta/h) u2
    dL/dy  = lambda + J(y)^T u1 + J(y*)^T u2 + (J'(y)[g1])^T u1 + (J'(y)[g2])^T u2
    dL/dlnA += u1^T (dS/dlnA(y) + (dS/dlnA)'(y)[g1]) + u2^T (dS/dlnA(y*) + (dS/dlnA)'(y)[g2])

where F'(y)[v] is the derivative of F at y in direction v (the second-derivative terms: the
iteration matrix depends on y).  Here they are taken by complex-step differentiation of the
analytic Jacobian and of dS/dlnA, which is exact to rounding.
"""

from __future__ import annotations

import numpy as np

from .integrate import ROS2_ALPHA, ROS2_BETA, ROS2_GAMMA, ROS2_M1, ROS2_M2
from .kinetics import dsource_dlnA, jacobian, source_terms
from .mechanism import R

# complex-step size of the directional derivatives (far below any rounding of the real part)
_CS_H = 1e-40


def _uniform_sequence(traj):
    n0 = len(traj[0])
    if any(len(t) != n0 for t in traj):
        return False
    dts = [d for _, d in traj[0]]
    return all([d for _, d in t] == dts for t in traj)


def be_tangent(mech, y0, traj, lnA=None, energy=0):
    """d y_N / d(lnA, y0) per cell, shape [nc, n, nr + n], along a recorded BE trajectory."""
    nc, n = y0.shape
    nr = mech.nr
    eye = np.eye(n)
    if _uniform_sequence(traj):
        s = np.zeros((nc, n, nr + n))
        s[:, :, nr:] = eye[None]
        for k in range(len(traj[0])):
            dt = traj[0][k][1]
            y = np.stack([traj[c][k][0] for c in range(nc)])
            A = eye[None] / dt - jacobian(mech, y, lnA, energy)
            rhs = s / dt
            rhs[:, :, :nr] += dsource_dlnA(mech, y, lnA, energy)
            s = np.linalg.solve(A, rhs)
        return s
    out = np.zeros((nc, n, nr + n))
    for c in range(nc):
        out[c] = be_tangent(mech, y0[c:c + 1], [traj[c]], lnA, energy)[0]
    return out


def be_adjoint(mech, lam_N, traj, lnA=None, energy=0):
    """Reverse sweep: returns (dL/dy0 [nc, n], dL/dlnA per cell [nc, nr]) given dL/dy_N."""
    nc, n = lam_N.shape
    eye = np.eye(n)
    if _uniform_sequence(traj):
        lam = np.array(lam_N, dtype=float, copy=True)
        g = np.zeros((nc, mech.nr))
        for k in reversed(range(len(traj[0]))):
            dt = traj[0][k][1]
            y = np.stack([traj[c][k][0] for c in range(nc)])
            A = eye[None] / dt - jacobian(mech, y, lnA, energy)
            mu = np.linalg.solve(np.transpose(A, (0, 2, 1)), lam[:, :, None])[:, :, 0]
            g += np.einsum("ci,cij->cj", mu, dsource_dlnA(mech, y, lnA, energy))
            lam = mu / dt
        return lam, g
    lam0 = np.zeros((nc, n))
    g = np.zeros((nc, mech.nr))
    for c in range(nc):
        l, gc = be_adjoint(mech, lam_N[c:c + 1], [traj[c]], lnA, energy)
        lam0[c], g[c] = l[0], gc[0]
    return lam0, g


def final_loss(mech, yN, w):
    """L = sum_c [T_N + sum_i w_ci Y_ci] and dL/dy_N ([nc, n])."""
    C = yN[:, 1:]
    rho = (C * mech.W[None, :]).sum(axis=1)
    Y = C * mech.W[None, :] / rho[:, None]
    L = float(yN[:, 0].sum() + (w * Y).sum())
    lam = np.zeros_like(yN)
    lam[:, 0] = 1.0
    # dY_i/dC_k = W_k (delta_ik - Y_i) / rho
    lam[:, 1:] = mech.W[None, :] / rho[:, None] * (w - (w * Y).sum(axis=1, keepdims=True))
    return L, lam


def init_map_vjp(mech, T0, p, Y0, lam0):
    """Pull dL/dy0 back through y0 = (T0, C(T0, p, Y0)): returns (dL/dT0, dL/dY0)."""
    Wbar = 1.0 / (Y0 / mech.W[None, :]).sum(axis=1)
    rho = p * Wbar / (R * T0)
    C = rho[:, None] * Y0 / mech.W[None, :]
    lamC = lam0[:, 1:]
    dT = lam0[:, 0] - (lamC * C).sum(axis=1) / T0
    s = (lamC * Y0 / mech.W[None, :]).sum(axis=1)
    dY = rho[:, None] / mech.W[None, :] * (lamC - (Wbar * s)[:, None])
    return dT, dY


# ----------------------------------------------------------------------------- Rosenbrock

def ros2_replay(mech, y0, steps, lnA=None, energy=0, keep=False):
    """Apply the recorded Rosenbrock steps of one cell: y0 [n], steps = step sizes in order.

    Every step is taken as given (no error control).  Works in complex arithmetic as well
    (complex y0 or lnA), which the complex-step pins use.  Returns the final state, or with
    ``keep`` the list of states before each step followed by the final one.
    """
    y = np.array(y0)[None, :]
    if lnA is not None and np.iscomplexobj(lnA):
        y = y.astype(complex)
    n = y.shape[1]
    eye = np.eye(n)
    states = []
    for h in steps:
        states.append(y[0].copy())
        G = eye / (ROS2_GAMMA * h) - jacobian(mech, y, lnA, energy)[0]
        g1 = np.linalg.solve(G, source_terms(mech, y, lnA, energy)[0])
        ys = y + ROS2_ALPHA * g1[None, :]
        g2 = np.linalg.solve(G, source_terms(mech, ys, lnA, energy)[0] + (ROS2_BETA / h) * g1)
        y = y + (ROS2_M1 * g1 + ROS2_M2 * g2)[None, :]
    if keep:
        states.append(y[0].copy())
        return states
    return y[0]


def _directional(f, y, v):
    """F'(y)[v] by complex step for a function of a [1, n] state."""
    return np.imag(f(y[None, :] + 1j * _CS_H * v[None, :])[0]) / _CS_H


def ros2_adjoint_cell(mech, lam_N, y0, steps, lnA=None, energy=0):
    """Reverse sweep of one cell's recorded Rosenbrock steps: returns (dL/dy0 [n], dL/dlnA [nr])."""
    states = ros2_replay(mech, y0, steps, lnA, energy, keep=True)
    n = len(lam_N)
    eye = np.eye(n)
    lam = np.array(lam_N, dtype=float, copy=True)
    g = np.zeros(mech.nr)
    jac = lambda yy: jacobian(mech, yy, lnA, energy)  # noqa: E731
    dsl = lambda yy: dsource_dlnA(mech, yy, lnA, energy)  # noqa: E731
    for k in reversed(range(len(steps))):
        y, h = states[k], steps[k]
        J = jac(y[None, :])[0]
        G = eye / (ROS2_GAMMA * h) - J
        g1 = np.linalg.solve(G, source_terms(mech, y[None, :], lnA, energy)[0])
        ys = y + ROS2_ALPHA * g1
        g2 = np.linalg.solve(G, source_terms(mech, ys[None, :], lnA, energy)[0] + (ROS2_BETA / h) * g1)
        Js = jac(ys[None, :])[0]
        u2 = np.linalg.solve(G.T, ROS2_M2 * lam)
        u1 = np.linalg.solve(G.T, ROS2_M1 * lam + ROS2_ALPHA * (Js.T @ u2) + (ROS2_BETA / h) * u2)
        dJ1 = _directional(jac, y, g1)
        dJ2 = _directional(jac, y, g2)
        g += u1 @ (dsl(y[None, :])[0] + _directional(dsl, y, g1)) \
            + u2 @ (dsl(ys[None, :])[0] + _directional(dsl, y, g2))
        lam = lam + J.T @ u1 + Js.T @ u2 + dJ1.T @ u1 + dJ2.T @ u2
    return lam, g


def ros2_adjoint(mech, lam_N, y0, histories, lnA=None, energy=0):
    """Per-cell reverse sweeps: histories[c] = list of accepted step sizes of cell c (or of
    (h, err) pairs as ``integrate_ros2(record=True)`` returns them).  Returns (dL/dy0 [nc, n],
    dL/dlnA per cell [nc, nr])."""
    nc, n = lam_N.shape
    lam0 = np.zeros((nc, n))
    g = np.zeros((nc, mech.nr))
    for c in range(nc):
        steps = [s[0] if isinstance(s, tuple) else s for s in histories[c]]
        lam0[c], g[c] = ros2_adjoint_cell(mech, lam_N[c], y0[c], steps, lnA, energy)
    return lam0, g
