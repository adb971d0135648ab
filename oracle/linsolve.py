"""Iterative linear solver of the oracle (paper Section 3.4): restarted GMRES with optional Jacobi
preconditioning -- TEST INFRASTRUCTURE ONLY.

GMRES (Saad and Schultz, 1986) minimises the residual over the Krylov subspace
K_j = span{r0, B r0, ..., B^(j-1) r0}.  Preconditioning is applied from the left as in the paper's
M^-1 A x = M^-1 b, with M = diag(A) (Jacobi: the reciprocals of the diagonal entries) or M = I, so
the residual that is minimised and tested is the preconditioned one, r = M^-1 (b - A x).

Steps of one cycle, from the current iterate x (x0 = 0):
  r0 = M^-1 (b - A x), beta = |r0|, v_1 = r0 / beta;
  Arnoldi with modified Gram-Schmidt: w = M^-1 A v_j; h_ij = (w, v_i), w -= h_ij v_i for i <= j;
  h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j};
  y_j = argmin |beta e_1 - Hbar_j y| (the (j+1) x j Hessenberg matrix), whose residual is
  |M^-1 (b - A (x + V_j y_j))|.  Two textbook ways to solve that small least-squares problem
  are offered: numpy.linalg.lstsq on Hbar_j (``lsq="lstsq"``), or Givens rotations applied to
  each new column of Hbar_j as it is formed, with |g_{j+1}| as the residual and back substitution
  on the rotated triangle (``lsq="givens"``).  They agree in exact arithmetic; on badly scaled
  systems their rounding differs visibly, which the tests use to measure how well the iterate is
  determined.
The solve stops when that residual is <= rtol |M^-1 b|, after max_iter iterations in all, or at a
happy breakdown (h_{j+1,j} = 0: the Krylov space is invariant and x + V_j y_j is exact).  After m
iterations without stopping the cycle restarts from x + V_m y_m.
"""

from __future__ import annotations

import numpy as np


def _givens_cycle_solve(H, beta, j):
    """min |beta e_1 - H[:j+2, :j+1] y| by Givens rotations (column by column) and back
    substitution; returns (y, residual)."""
    R = H[:j + 2, :j + 1].copy()
    g = np.zeros(j + 2)
    g[0] = beta
    for i in range(j + 1):
        den = np.hypot(R[i, i], R[i + 1, i])
        c, s = R[i, i] / den, R[i + 1, i] / den
        Ri, Ri1 = R[i, :].copy(), R[i + 1, :].copy()
        R[i, :], R[i + 1, :] = c * Ri + s * Ri1, -s * Ri + c * Ri1
        g[i], g[i + 1] = c * g[i] + s * g[i + 1], -s * g[i] + c * g[i + 1]
    y = np.zeros(j + 1)
    for i in range(j, -1, -1):
        y[i] = (g[i] - R[i, i + 1:j + 1] @ y[i + 1:]) / R[i, i]
    return y, abs(g[j + 1])


PRECOND_NONE, PRECOND_JACOBI, PRECOND_GS = 0, 1, 2


def _forward_substitution(L, v):
    """Solve L w = v for lower-triangular L (row by row)."""
    w = np.zeros_like(v)
    for i in range(L.shape[0]):
        w[i] = (v[i] - L[i, :i] @ w[:i]) / L[i, i]
    return w


def gmres(A, b, m, rtol, max_iter, precond=PRECOND_JACOBI, lsq="lstsq"):
    """Restarted GMRES(m) for one system A x = b ([n, n], [n]).  Returns (x, iterations, converged).
    m <= 0 means m = n (no restart); ``precond``: PRECOND_NONE (or False), PRECOND_JACOBI (or True),
    PRECOND_GS; ``lsq`` picks the least-squares solve ("lstsq" or "givens")."""
    A = np.asarray(A, dtype=float)
    b = np.asarray(b, dtype=float)
    n = b.shape[0]
    m = n if m <= 0 else min(m, n)
    precond = int(precond)
    if precond == PRECOND_GS:
        L = np.tril(A)
        B = np.stack([_forward_substitution(L, A[:, k]) for k in range(n)], axis=1)   # M^-1 A
        c = _forward_substitution(L, b)                                               # M^-1 b
    else:
        dinv = 1.0 / np.diag(A) if precond == PRECOND_JACOBI else np.ones(n)
        B = dinv[:, None] * A                       # M^-1 A
        c = dinv * b                                # M^-1 b
    target = rtol * np.linalg.norm(c)
    x = np.zeros(n)
    its = 0
    if np.linalg.norm(c) == 0.0:
        return x, 0, True
    while its < max_iter:
        r0 = c - B @ x
        beta = np.linalg.norm(r0)
        if beta <= target:
            return x, its, True
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        V[:, 0] = r0 / beta
        y = np.zeros(0)
        for j in range(m):
            w = B @ V[:, j]
            for i in range(j + 1):
                H[i, j] = w @ V[:, i]
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            if lsq == "givens":
                y, res = _givens_cycle_solve(H, beta, j)
            else:
                e1 = np.zeros(j + 2)
                e1[0] = beta
                y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
                res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            breakdown = H[j + 1, j] == 0.0
            if res <= target or breakdown or its >= max_iter:
                return x + V[:, :j + 1] @ y, its, bool(res <= target or breakdown)
            V[:, j + 1] = w / H[j + 1, j]
        x = x + V[:, :m] @ y
    return x, its, False
