"""Rates of progress, source terms and their analytic Jacobian (paper Sections 2.2 and 3.2).

State per cell: y = (T, C_1..C_ns) (eq. extracted_problem), arrays of shape
[nc, n] with n = ns + 1.  ``lnA`` is the per-reaction ln of the
(high-pressure) Arrhenius prefactor; for falloff reactions the low-pressure
prefactor moves with it, so P_r does not depend on lnA.

Definitions followed (all in SI-kmol units):

* k_A = exp(ln A + b ln T - theta / T)                         (Arrhenius, log form)
* third body: k_f = [M] k_A, [M] = sum_i alpha_ij C_i             (eqs. third_body, TB_optimization)
* falloff: k_f = k_inf * P_r / (1 + P_r) * F, P_r = k_0 [M] / k_inf  (eq. falloff-reaction)
* Troe F from F_cent, c, n, f1 (eq. f_and_fcent); SRI F = d [a exp(-b/T) + exp(-T/c)]^X T^e with
  X = 1/(1 + (log10 P_r)^2) (the SRI form Section 2.2 lists beside Troe); Lindemann F = 1
* P-log: ln k interpolated linearly in ln p between tabulated Arrhenius sets, p = R T sum C
* K_j = exp(-sum_i nu_ij g_i/RT) (p_ref / RT)^(sum_i nu_ij),  k_r = k_f / K_j  (eqs. reverse_rate,
  equilibrium-constant)
* q_j = k_f prod C^nu_f - k_r prod C^nu_r; omega_i = sum_j nu_ij q_j
* omega_T = -sum H_i omega_i / sum C_i Cp_i at constant pressure (Appendix B, eq.
  temperature_source_h) or -sum U_i omega_i / sum C_i Cv_i at constant volume (eq.
  temperature_source); the denominators are volumetric heat capacities.
* constant-pressure reactor with dilatation (energy = CONST_P_REACTOR): the same omega_T, and the
  concentrations also follow the density change.  With C_i = rho Y_i / W_i, dY_i/dt = W_i omega_i /
  rho and rho = p Wbar / (R T) at fixed p, d ln rho / dt = -g with g = sum_j omega_j / sum_j C_j +
  omega_T / T, so dC_i/dt = omega_i - C_i g.  (Appendix B's source terms keep dC_i/dt = omega_i,
  i.e. they neglect this term; the reactor form keeps p = R T sum C and the mass-specific
  enthalpy sum C_i H_i / rho constant.)
"""

from __future__ import annotations

import numpy as np

from .mechanism import R
from .thermo import nasa7_molar

LN10 = np.log(10.0)
CONST_P, CONST_V, CONST_P_REACTOR = 0, 1, 2


def _conc_product(C, stoich):
    """prod_i C_i^nu_i with integer exponents, by repeated multiplication."""
    out = np.ones(C.shape[0], dtype=C.dtype)
    for i, v in stoich.items():
        for _ in range(v):
            out = out * C[:, i]
    return out


def _conc_product_derivs(C, stoich):
    """d/dC_k of prod_i C_i^nu_i for each participant k: dict k -> array."""
    out = {}
    for k, vk in stoich.items():
        d = vk * np.ones(C.shape[0], dtype=C.dtype)
        for _ in range(vk - 1):
            d = d * C[:, k]
        for i, v in stoich.items():
            if i != k:
                for _ in range(v):
                    d = d * C[:, i]
        out[k] = d
    return out


def _troe(rx, T, Pr, magnitude=False):
    """Troe broadening: returns (F, dlog10F/dlog10Pr, dlog10F/dT at fixed Pr).

    With ``magnitude`` also returns the term-wise absolute size of the T derivative.
    """
    alpha, T3, T1, T2 = rx.troe
    e3 = np.exp(-T / T3)
    e1 = np.exp(-T / T1)
    Fc = (1.0 - alpha) * e3 + alpha * e1
    dFc = -(1.0 - alpha) / T3 * e3 - alpha / T1 * e1
    dFc_mag = np.abs(1.0 - alpha) / T3 * np.abs(e3) + abs(alpha) / T1 * np.abs(e1)
    if T2 is not None:
        e2 = np.exp(-T2 / T)
        Fc = Fc + e2
        dFc = dFc + T2 / (T * T) * e2
        dFc_mag = dFc_mag + np.abs(T2 / (T * T) * e2)
    Fc = np.where(np.real(Fc) > 1e-300, Fc, 1e-300)
    L = np.log(Fc) / LN10
    Prc = np.where(np.real(Pr) > 1e-300, Pr, 1e-300)
    lPr = np.log(Prc) / LN10
    c = -0.4 - 0.67 * L
    nn = 0.75 - 1.27 * L
    x = lPr + c
    den = nn - 0.14 * x
    f1 = x / den
    log10F = L / (1.0 + f1 * f1)
    F = np.exp(LN10 * log10F)
    # derivatives of log10 F
    g = 1.0 / (1.0 + f1 * f1)
    dlogF_df1 = -L * 2.0 * f1 * g * g
    df1_dx = nn / (den * den)
    dlogF_dlPr = dlogF_df1 * df1_dx
    df1_dL = (-0.67 * nn + 1.27 * x) / (den * den)
    dlogF_dL = g + dlogF_df1 * df1_dL
    dL_dT = dFc / (Fc * LN10)
    if not magnitude:
        return F, dlogF_dlPr, dlogF_dL * dL_dT
    df1_dL_mag = (0.67 * np.abs(nn) + 1.27 * np.abs(x)) / np.abs(den * den)
    mag = (np.abs(g) + np.abs(dlogF_df1) * df1_dL_mag) * dFc_mag / (np.abs(Fc) * LN10)
    return F, dlogF_dlPr, dlogF_dL * dL_dT, mag


def _sri(rx, T, Pr):
    """SRI broadening F = d [a exp(-b/T) + exp(-T/c)]^X T^e, X = 1/(1 + (log10 P_r)^2).

    Returns (F, dlog10F/dlog10Pr, dlog10F/dT at fixed Pr, term-wise size of the T derivative).
    """
    a, b, c, d, e = rx.sri
    ea = np.exp(-b / T)
    ec = np.exp(-T / c)
    B = a * ea + ec
    B = np.where(np.real(B) > 1e-300, B, 1e-300)
    Prc = np.where(np.real(Pr) > 1e-300, Pr, 1e-300)
    lPr = np.log(Prc) / LN10
    X = 1.0 / (1.0 + lPr * lPr)
    log10F = np.log(d) / LN10 + X * np.log(B) / LN10 + e * np.log(T) / LN10
    F = np.exp(LN10 * log10F)
    dlogF_dlPr = (np.log(B) / LN10) * (-2.0 * lPr * X * X)
    dB = a * b / (T * T) * ea - ec / c
    dlogF_dT = (X * dB / B + e / T) / LN10
    dB_mag = np.abs(a) * b / np.abs(T * T) * np.abs(ea) + np.abs(ec) / c
    mag = (np.abs(X) * dB_mag / np.abs(B) + abs(e) / np.abs(T)) / LN10
    return F, dlogF_dlPr, dlogF_dT, mag


def _plog_rate(rx, j, T, lnT, invT, C, lnA):
    """P-log (Section 2.2, other pressure-dependent forms): ln k is interpolated linearly in ln p
    between the Arrhenius sets of the two tabulated pressures around p = R T sum_i C_i, and held
    at the end sets outside the table.  Every set carries the same ln A shift as the reaction's
    parameter lnA[j] (which is ln A of the lowest-pressure set).
    Returns (kf, dlnkf_dT, M = sum C, dlnkf_dM, |dlnkf_dT| term-wise, |dlnkf_dM|)."""
    M = C.sum(axis=1)
    lnp = np.log(R * T * M)
    sets = rx.plog
    lnk = [lnA[j] + (lA - rx.lnA) + b * lnT - th * invT for _, lA, b, th in sets]
    # term-wise size of each ln k_i: the rounding scale of a difference ln k_{i+1} - ln k_i
    lnk_mag = [np.abs(lnA[j] + (lA - rx.lnA)) + abs(b) * np.abs(lnT) + abs(th) * np.abs(invT)
               for _, lA, b, th in sets]
    dk = [(b + th * invT) * invT for _, _, b, th in sets]
    dk_mag = [(abs(b) + abs(th) * np.abs(invT)) * np.abs(invT) for _, _, b, th in sets]
    lr = np.real(lnp)
    out_k = lnk[0] + 0.0 * lnp
    out_dT = dk[0] + 0.0 * lnp
    out_dp = 0.0 * lnp
    out_dp_mag = 0.0 * lr
    out_mag = dk_mag[0] + 0.0 * lr
    for i in range(len(sets) - 1):
        l0, l1 = sets[i][0], sets[i + 1][0]
        inside = (lr > l0) & (lr <= l1)
        w = (lnp - l0) / (l1 - l0)
        out_k = np.where(inside, lnk[i] + w * (lnk[i + 1] - lnk[i]), out_k)
        out_dT = np.where(inside, (1.0 - w) * dk[i] + w * dk[i + 1], out_dT)
        out_dp = np.where(inside, (lnk[i + 1] - lnk[i]) / (l1 - l0), out_dp)
        out_dp_mag = np.where(inside, (lnk_mag[i + 1] + lnk_mag[i]) / (l1 - l0), out_dp_mag)
        out_mag = np.where(inside, np.abs(1.0 - w) * dk_mag[i] + np.abs(w) * dk_mag[i + 1], out_mag)
    above = lr > sets[-1][0]
    out_k = np.where(above, lnk[-1], out_k)
    out_dT = np.where(above, dk[-1], out_dT)
    out_mag = np.where(above, dk_mag[-1], out_mag)
    # d ln p / dT = 1/T and d ln p / dC_k = 1/sum C at fixed C and T.  The magnitudes of the
    # p-derivative take the term-wise size of the two ln k it differences (they nearly cancel
    # where two tabulated sets cross).
    dlnkf_dT = out_dT + out_dp * invT
    mag_T = out_mag + out_dp_mag * np.abs(invT)
    return np.exp(out_k), dlnkf_dT, M, out_dp / M, mag_T, out_dp_mag / np.abs(M)


def _forward_rate(mech, rx, j, T, lnT, invT, C, lnA):
    """k_f and the pieces needed by the Jacobian.

    Returns (kf, dlnkf_dT, M, dlnkf_dM, |dlnkf_dT| term-wise, |dlnkf_dM| term-wise);
    M is None for elementary reactions.
    """
    if rx.kind == "plog":
        return _plog_rate(rx, j, T, lnT, invT, C, lnA)
    lnk = lnA[j] + rx.b * lnT - rx.theta * invT
    dlnk_dT = (rx.b + rx.theta * invT) * invT
    dlnk_dT_mag = (abs(rx.b) + abs(rx.theta) * np.abs(invT)) * np.abs(invT)
    if rx.kind == "elementary":
        return np.exp(lnk), dlnk_dT, None, None, dlnk_dT_mag, None
    M = C @ rx.eff                                     # sum_i alpha_ij C_i
    if rx.kind == "three-body":
        return M * np.exp(lnk), dlnk_dT, M, 1.0 / M, dlnk_dT_mag, 1.0 / np.abs(M)
    # falloff: k_0 carries the same ln A shift as k_inf
    lnk0 = lnA[j] + (rx.lnA0 - rx.lnA) + rx.b0 * lnT - rx.theta0 * invT
    kinf = np.exp(lnk)
    Pr = np.exp(lnk0 - lnk) * M
    dlnPr_dT = ((rx.b0 - rx.b) + (rx.theta0 - rx.theta) * invT) * invT
    dlnPr_dT_mag = (abs(rx.b0 - rx.b) + abs(rx.theta0 - rx.theta) * np.abs(invT)) * np.abs(invT)
    if rx.troe is not None:
        F, dlF_dlPr, dlF_dT, dlF_dT_mag = _troe(rx, T, Pr, magnitude=True)
    elif rx.sri is not None:
        F, dlF_dlPr, dlF_dT, dlF_dT_mag = _sri(rx, T, Pr)
    else:
        F, dlF_dlPr, dlF_dT, dlF_dT_mag = 1.0, 0.0, 0.0, 0.0
    kf = kinf * Pr / (1.0 + Pr) * F
    dlnkf_dT = dlnk_dT + dlnPr_dT / (1.0 + Pr) + LN10 * dlF_dT + dlF_dlPr * dlnPr_dT
    # d ln kf / d M  (P_r proportional to M)
    dlnkf_dM = (1.0 / (1.0 + Pr) + dlF_dlPr) / M
    a1 = np.abs(1.0 / (1.0 + Pr))
    mag_T = dlnk_dT_mag + dlnPr_dT_mag * a1 + LN10 * dlF_dT_mag + np.abs(dlF_dlPr) * dlnPr_dT_mag
    mag_M = (a1 + np.abs(dlF_dlPr)) / np.abs(M)
    return kf, dlnkf_dT, M, dlnkf_dM, mag_T, mag_M


def _lnKc(mech, j, T, lnT, g_RT):
    nu = mech.nu[:, j]
    dnu = nu.sum()
    return -(g_RT @ nu) + dnu * (np.log(mech.p_ref / R) - lnT)


def _prepare(mech, y, lnA):
    y = np.asarray(y)
    if y.ndim == 1:
        y = y[None, :]
    T = y[:, 0]
    C = y[:, 1:]
    lnA = mech.lnA_default if lnA is None else np.asarray(lnA)
    return y, T, C, lnA


def rates_of_progress(mech, y, lnA=None):
    """q_j [nc, nr] plus the forward/reverse parts (Rf, Rr) and thermo (eq. chemical-reaction-rate-of-progress)."""
    y, T, C, lnA = _prepare(mech, y, lnA)
    lnT = np.log(T)
    invT = 1.0 / T
    cp_R, h_RT, s_R, g_RT, dcp_R = nasa7_molar(mech, T)
    nc = y.shape[0]
    q = np.zeros((nc, mech.nr), dtype=y.dtype)
    Rf = np.zeros_like(q)
    Rr = np.zeros_like(q)
    for j, rx in enumerate(mech.reactions):
        kf = _forward_rate(mech, rx, j, T, lnT, invT, C, lnA)[0]
        Rf[:, j] = kf * _conc_product(C, rx.reactants)
        if rx.reversible:
            kr = kf / np.exp(_lnKc(mech, j, T, lnT, g_RT))
            Rr[:, j] = kr * _conc_product(C, rx.products)
        q[:, j] = Rf[:, j] - Rr[:, j]
    return q, Rf, Rr, (cp_R, h_RT, s_R, g_RT, dcp_R)


def _temperature_weights(h_RT, cp_R, energy):
    """(enthalpy-like weights H_i/RT, heat-capacity weights Cp_i/R) for the chosen energy mode."""
    if energy in (CONST_P, CONST_P_REACTOR):
        return h_RT, cp_R
    return h_RT - 1.0, cp_R - 1.0   # U/RT = H/RT - 1, Cv/R = Cp/R - 1


def _dilatation_rate(S0, T, C):
    """g = sum_j omega_j / sum_j C_j + omega_T / T (so that d ln rho/dt = -g at constant p)."""
    return S0[:, 1:].sum(axis=1) / C.sum(axis=1) + S0[:, 0] / T


def source_terms(mech, y, lnA=None, energy=CONST_P):
    """S(y) = (omega_T, omega_1..omega_ns), shape [nc, n]; for CONST_P_REACTOR the species
    entries are omega_i - C_i g."""
    if energy == CONST_P_REACTOR:
        yy, T, C, _ = _prepare(mech, y, lnA)
        S0 = source_terms(mech, y, lnA, CONST_P)
        S = S0.copy()
        S[:, 1:] -= C * _dilatation_rate(S0, T, C)[:, None]
        return S
    y, T, C, lnA = _prepare(mech, y, lnA)
    q, _, _, th = rates_of_progress(mech, y, lnA)
    cp_R, h_RT = th[0], th[1]
    omega = q @ mech.nu.T                        # omega_i = sum_j nu_ij q_j
    hw, cw = _temperature_weights(h_RT, cp_R, energy)
    N = (hw * omega).sum(axis=1)
    D = (C * cw).sum(axis=1)
    omega_T = -T * N / D
    return np.concatenate([omega_T[:, None], omega], axis=1)


def source_sum_scale(mech, y, lnA=None, energy=CONST_P):
    """Magnitude of the sums that form S: sum_j |nu_ij| (|R_f,j| + |R_r,j|) per species and the
    matching T term.

    Used to express floating-point tolerances relative to the size of the terms that
    are summed (the bound on summation error), not to the possibly cancelled result.  Each
    q_j = R_f - R_r is itself such a sum: near partial equilibrium R_f and R_r nearly cancel, so
    the scale takes both rates, not |q_j|.
    """
    y, T, C, lnA = _prepare(mech, y, lnA)
    _, Rf, Rr, th = rates_of_progress(mech, y, lnA)
    cp_R, h_RT = th[0], th[1]
    mag = (np.abs(Rf) + np.abs(Rr)) @ np.abs(mech.nu.T)
    hw, cw = _temperature_weights(h_RT, cp_R, energy)
    D = (C * cw).sum(axis=1)
    magT = np.abs(T) * (np.abs(hw) * mag).sum(axis=1) / np.abs(D)
    if energy == CONST_P_REACTOR:
        # the dilatation term C_i g sums the species rates and omega_T / T
        gm = mag.sum(axis=1) / np.abs(C.sum(axis=1)) + magT / np.abs(T)
        mag = mag + np.abs(C) * gm[:, None]
    return np.concatenate([magT[:, None], mag], axis=1)


def jacobian(mech, y, lnA=None, energy=CONST_P, magnitude=False):
    """Analytic J = dS/dy, shape [nc, n, n], index 0 = T (eq. derivative_matrices_temp_evol).

    Built reaction by reaction from d q_j / d(T, C) (mass action, third-body and falloff
    chain rules, d ln K / dT = (sum_i nu_ij h_i/RT - sum_i nu_ij) / T), then the T row by
    the quotient rule applied to omega_T = -T N / D.

    With ``magnitude`` also returns M (same shape): every entry recomputed with the absolute
    value of each term it sums, the scale that bounds the rounding error of that entry.

    CONST_P_REACTOR: the species rows of dS/dy for S_i = omega_i - C_i g are J_ik - delta_ik g -
    C_i dg/dy_k with dg/dy_k = (sum_j J_jk) / sum C - [k >= 1] sum omega / (sum C)^2 + J_0k / T -
    [k = 0] omega_T / T^2 (J: the constant-pressure Jacobian, sums over the species rows).
    """
    if energy == CONST_P_REACTOR:
        yy, T, C, _ = _prepare(mech, y, lnA)
        res = jacobian(mech, y, lnA, CONST_P, magnitude)
        J0, M0 = res if magnitude else (res, None)
        S0 = source_terms(mech, y, lnA, CONST_P)
        c, Om = C.sum(axis=1), S0[:, 1:].sum(axis=1)
        g = Om / c + S0[:, 0] / T
        dg = J0[:, 1:, :].sum(axis=1) / c[:, None] + J0[:, 0, :] / T[:, None]
        dg[:, 1:] -= (Om / c ** 2)[:, None]
        dg[:, 0] -= S0[:, 0] / T ** 2
        J = J0.copy()
        J[:, 1:, :] -= C[:, :, None] * dg[:, None, :]
        J[:, 1:, 1:] -= g[:, None, None] * np.eye(mech.ns)[None]
        if not magnitude:
            return J
        sc = source_sum_scale(mech, y, lnA, CONST_P)
        gm = sc[:, 1:].sum(axis=1) / np.abs(c) + sc[:, 0] / np.abs(T)
        dgm = M0[:, 1:, :].sum(axis=1) / np.abs(c)[:, None] + M0[:, 0, :] / np.abs(T)[:, None]
        dgm[:, 1:] += (sc[:, 1:].sum(axis=1) / c ** 2)[:, None]
        dgm[:, 0] += sc[:, 0] / T ** 2
        Mg = M0.copy()
        Mg[:, 1:, :] += np.abs(C)[:, :, None] * dgm[:, None, :]
        Mg[:, 1:, 1:] += gm[:, None, None] * np.eye(mech.ns)[None]
        return J, Mg
    y, T, C, lnA = _prepare(mech, y, lnA)
    nc, n, ns = y.shape[0], mech.n, mech.ns
    lnT = np.log(T)
    invT = 1.0 / T
    cp_R, h_RT, s_R, g_RT, dcp_R = nasa7_molar(mech, T)
    dq = np.zeros((nc, mech.nr, n), dtype=y.dtype)   # d q_j / d y_k
    dqm = np.zeros((nc, mech.nr, n)) if magnitude else None
    q = np.zeros((nc, mech.nr), dtype=y.dtype)
    for j, rx in enumerate(mech.reactions):
        kf, dlnkf_dT, M, dlnkf_dM, mag_T, mag_M = _forward_rate(mech, rx, j, T, lnT, invT, C, lnA)
        Pf = _conc_product(C, rx.reactants)
        dPf = _conc_product_derivs(C, rx.reactants)
        Rf = kf * Pf
        Rr = np.zeros_like(Rf)
        dlnKc_dT = np.zeros_like(Rf)
        dlnKc_dT_mag = 0.0
        if rx.reversible:
            Kc = np.exp(_lnKc(mech, j, T, lnT, g_RT))
            kr = kf / Kc
            Pr_ = _conc_product(C, rx.products)
            Rr = kr * Pr_
            nu = mech.nu[:, j]
            dlnKc_dT = (h_RT @ nu - nu.sum()) * invT
            dlnKc_dT_mag = (np.abs(h_RT) @ np.abs(nu) + abs(nu.sum())) * np.abs(invT)
            for k, d in _conc_product_derivs(C, rx.products).items():
                dq[:, j, 1 + k] -= kr * d
                if magnitude:
                    dqm[:, j, 1 + k] += np.abs(kr * d)
        for k, d in dPf.items():
            dq[:, j, 1 + k] += kf * d
            if magnitude:
                dqm[:, j, 1 + k] += np.abs(kf * d)
        qj = Rf - Rr
        q[:, j] = qj
        dq[:, j, 0] = qj * dlnkf_dT + Rr * dlnKc_dT
        if magnitude:
            dqm[:, j, 0] = (np.abs(Rf) + np.abs(Rr)) * mag_T + np.abs(Rr) * dlnKc_dT_mag
        if M is not None:
            # k_f depends on C through [M] = sum_i alpha_ij C_i
            dq[:, j, 1:] += (qj * dlnkf_dM)[:, None] * rx.eff[None, :]
            if magnitude:
                dqm[:, j, 1:] += ((np.abs(Rf) + np.abs(Rr)) * mag_M)[:, None] * np.abs(rx.eff)[None, :]
    J = np.zeros((nc, n, n), dtype=y.dtype)
    J[:, 1:, :] = np.einsum("ij,cjk->cik", mech.nu, dq)
    omega = q @ mech.nu.T
    hw, cw = _temperature_weights(h_RT, cp_R, energy)
    N = (hw * omega).sum(axis=1)
    D = (C * cw).sum(axis=1)
    a = T * N / (D * D)
    J[:, 0, 0] = -((cw * omega).sum(axis=1) + T * (hw * J[:, 1:, 0]).sum(axis=1)) / D \
        + a * (C * dcp_R).sum(axis=1)
    J[:, 0, 1:] = -T[:, None] * np.einsum("ci,cik->ck", hw, J[:, 1:, 1:]) / D[:, None] + a[:, None] * cw
    if not magnitude:
        return J
    Mg = np.zeros((nc, n, n))
    Mg[:, 1:, :] = np.einsum("ij,cjk->cik", np.abs(mech.nu), dqm)
    omm = np.abs(q) @ np.abs(mech.nu.T)
    Nm = (np.abs(hw) * omm).sum(axis=1)
    am = np.abs(T) * Nm / (D * D)
    Mg[:, 0, 0] = ((np.abs(cw) * omm).sum(axis=1) + np.abs(T) * (np.abs(hw) * Mg[:, 1:, 0]).sum(axis=1)) / np.abs(D) \
        + am * (np.abs(C) * np.abs(dcp_R)).sum(axis=1)
    Mg[:, 0, 1:] = np.abs(T)[:, None] * np.einsum("ci,cik->ck", np.abs(hw), Mg[:, 1:, 1:]) / np.abs(D)[:, None] \
        + am[:, None] * np.abs(cw)
    return J, Mg


def jacobian_complex_step(mech, y, lnA=None, energy=CONST_P, h=1e-40):
    """dS/dy by complex-step differentiation of ``source_terms`` (exact to rounding; a test pin)."""
    y = np.atleast_2d(np.asarray(y, dtype=float))
    nc, n = y.shape
    J = np.zeros((nc, n, n))
    for k in range(n):
        yc = y.astype(complex)
        yc[:, k] += 1j * h
        J[:, :, k] = np.imag(source_terms(mech, yc, lnA, energy)) / h
    return J


def dsource_dlnA(mech, y, lnA=None, energy=CONST_P):
    """dS/d lnA_j, shape [nc, n, nr]: lnA_j scales k_f and k_r (and k_0, k_inf) alike, so
    d q_j / d lnA_j = q_j, d omega_i / d lnA_j = nu_ij q_j and the T row follows omega_T (with the
    dilatation term, the species rows also subtract C_i dg/dlnA_j)."""
    if energy == CONST_P_REACTOR:
        yy, T, C, _ = _prepare(mech, y, lnA)
        P = dsource_dlnA(mech, y, lnA, CONST_P)
        dg = P[:, 1:, :].sum(axis=1) / C.sum(axis=1)[:, None] + P[:, 0, :] / T[:, None]
        P = P.copy()
        P[:, 1:, :] -= C[:, :, None] * dg[:, None, :]
        return P
    y, T, C, lnA = _prepare(mech, y, lnA)
    q, _, _, th = rates_of_progress(mech, y, lnA)
    cp_R, h_RT = th[0], th[1]
    hw, cw = _temperature_weights(h_RT, cp_R, energy)
    D = (C * cw).sum(axis=1)
    dom = mech.nu[None, :, :] * q[:, None, :]          # [nc, ns, nr]
    dT = -T[:, None] * np.einsum("ci,cij->cj", hw, dom) / D[:, None]
    return np.concatenate([dT[:, None, :], dom], axis=1)
