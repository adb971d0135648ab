"""Forward (tangent) and reverse (discrete adjoint) sensitivities of the backward-Euler map.

Each accepted (sub)step of size dt solves F(y', y, theta) = (y' - y)/dt - S(y', theta) = 0.
With A = dF/dy' = I/dt - J(y'):

* tangent:  A s' = s / dt + dS/dtheta(y')                     (s = dy/dtheta)
* adjoint:  A^T mu = lambda',  lambda = mu / dt,  g_theta += mu^T dS/dtheta(y')

theta = (ln A_1..ln A_nr, y0).  The loss of the differentiation workload is
L = sum_cells [T_N + sum_i w_i Y_i(y_N)] with Y_i = W_i C_i / sum_k W_k C_k, and the
initial state comes from (T0, p, Y0) through rho0 = p Wbar/(R T0), C_i = rho0 Y_i / W_i.
"""

from __future__ import annotations

import numpy as np

from .kinetics import dsource_dlnA, jacobian
from .mechanism import R


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
