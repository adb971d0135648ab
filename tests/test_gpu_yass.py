"""GPU: YASS (Appendix A.4, persistent form) with the LU and the GMRES solve (Section 3.4)
against the oracle, cell by cell.

Statuses, accepted substeps and rejected attempts must equal the oracle's (they are decided by
max(|dT|/T, max |dY|) <= alpha, which flips only if the norm lands within rounding of alpha).
Krylov iteration counts are sums over a cell's attempts of per-solve counts whose stopping test,
|g_{j+1}| <= rtol |M^-1 b|, is taken from Givens rotations on the GPU and from a least-squares
residual in the oracle: they must agree exactly for at least 90 % of the cells and within one per
attempt elsewhere.

States with LU: within 1e-8 (relative, species as mass fractions).  States with GMRES: a GMRES
iterate stopped by its tolerance is fixed only up to that residual, and on these badly scaled
systems (T next to concentrations of 1e-8; modified Gram-Schmidt loses orthogonality and the
small Hessenberg least-squares problem is ill-conditioned) rounding alone moves the integrated
states by 1e-12 .. 1e-6 depending on the mechanism and options.  The oracle shows it: an ulp-level
change of its input, or solving its Hessenberg problems by Givens rotations instead of LAPACK
lstsq (both exact in exact arithmetic), moves its states that much.  The bar is derived from that
sensitivity: 10 x the largest such change (at least 1e-8), over the cells whose counters these
variations leave unchanged (Krylov counts within one per attempt; at least 90 % of the cells),
and only those cells are compared.  The others hold a solve whose explicitly recomputed residual
stays at its rounding floor above the target, where the two formulations part (one runs to
krylov_max_iter, the other stops) and the states can differ by O(1) in a minor species.  (krylov_rtol = 0,
iterating past the rounding floor, is ill-posed: there the oracle's own states move by up to 1e-1
under ulp perturbations.)

Cases: the backward-Euler workload's states at the paper's YASS step (1e-7 s, Table 5) and at
2 x 1e-6 s (substep halving active) in both energy modes, a tighter alpha, GMRES with Jacobi
preconditioning (constant pressure with the density held, constant volume, the constant-pressure
reactor, a tighter alpha, restarted GMRES(4)), with Gauss-Seidel preconditioning (the same three
energy modes) and without, the Rosenbrock
workload's hot states, the h_min failure and the attempt budget, argument errors, and sampled
cells of the 1024-cell workload over its 2e-5 s at the paper's step with the autotuned launch.
"""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
from oracle.integrate import IntegratorOptions
from synth.states import STATE_CONFIGS, sample_config, sample_states

from _gpu import dev_soa, gpu_mechanism, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu

MECHS = ["tiny_5_6", "tiny_8_14", "h2like_10_27"]


@pytest.fixture(scope="module", params=MECHS)
def mechs(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


def _gpu_opts(kw):
    """Oracle options -> library options (the same names; krylov_lsq is the oracle's alone)."""
    return {k: v for k, v in kw.items() if k != "krylov_lsq"}


def _run(gm, y0, dt, n_steps, ld=None, **kw):
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_YASS, default_options
    nc = y0.shape[0]
    ld = ld or nc + 7
    y = dev_soa(y0, ld)
    st = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, ld), dtype=torch.int32, device="cuda")
    opts = default_options(method=CHEM_YASS, dt=dt, n_steps=n_steps, form=CHEM_PERSISTENT, **_gpu_opts(kw))
    gm.chem_integrate(nc, ld, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    return host_aos(y, nc), st.cpu().numpy()[:nc], cnt.cpu().numpy()[:, :nc]


def _check(om, ref, got, st, cnt, stable=None, krylov_alt=None):
    """Counters (on the cells in ``stable``, default all; Krylov counts against the nearer of the
    oracle's two GMRES formulations when ``krylov_alt`` is given) and the largest state error."""
    stable = np.ones(len(st), dtype=bool) if stable is None else stable
    np.testing.assert_array_equal(st[stable], ref["status"][stable])
    np.testing.assert_array_equal(cnt[0][stable], ref["accepted"][stable])
    np.testing.assert_array_equal(cnt[1][stable], ref["rejected"][stable])
    d = np.abs(cnt[2].astype(np.int64) - ref["krylov"])
    if krylov_alt is not None:
        d = np.minimum(d, np.abs(cnt[2].astype(np.int64) - krylov_alt))
    d = d[stable]
    attempts = (ref["accepted"] + ref["rejected"])[stable]
    assert (d == 0).mean() >= 0.9 and np.all(d <= attempts), (cnt[2], ref["krylov"])
    err = integrated_state_error(om, got, ref["y"])
    return err[stable].max()


def _sensitivity(om, y0, dt, n_steps, opt, ref):
    """Largest change of the oracle's states under ulp-level perturbations of the input and under
    the other least-squares solve of the GMRES Hessenberg problem (Givens rotations instead of
    LAPACK lstsq), the cells whose counters these leave unchanged, and the Krylov counts of the
    Givens formulation.  (Where a system's explicitly recomputed residual stays at its rounding
    floor above the target, the lstsq formulation runs to krylov_max_iter while the Givens
    residual estimate drops below the target and stops.)"""
    rng = np.random.default_rng(77)
    spread = 0.0
    stable = np.ones(y0.shape[0], dtype=bool)
    runs = [(y0 * (1.0 + rng.integers(-2, 3, size=y0.shape) * np.finfo(float).eps), opt) for _ in range(3)]
    runs.append((y0, dataclasses.replace(opt, krylov_lsq="givens")))
    for yp, op in runs:
        with np.errstate(all="ignore"):
            rp = oracle.integrate_yass(om, yp, dt, n_steps, opt=op)
        stable &= (rp["status"] == ref["status"]) & (rp["accepted"] == ref["accepted"]) & \
            (rp["rejected"] == ref["rejected"]) & \
            (np.abs(rp["krylov"] - ref["krylov"]) <= ref["accepted"] + ref["rejected"])
        spread = max(spread, integrated_state_error(om, rp["y"], ref["y"])[stable].max())
    return spread, stable, rp["krylov"]


CASES = {
    # name: (state config, cells, dt, n_steps, energy, options)
    "lu_paper_step": ("be_small", 150, 1e-7, 1, 0, {}),
    "lu_halving": ("be_small", 150, 2e-6, 2, 0, {}),
    "lu_halving_cv": ("be_small", 150, 2e-6, 2, 1, {}),
    "lu_tight_alpha": ("be_small", 150, 1e-6, 1, 0, dict(yass_alpha=0.01)),
    "gmres_jacobi": ("be_small", 150, 2e-6, 2, 0, dict(linear_solver=1)),
    "gmres_jacobi_cv": ("be_small", 150, 2e-6, 2, 1, dict(linear_solver=1)),
    "gmres_jacobi_tight_alpha": ("be_small", 150, 1e-6, 1, 0, dict(linear_solver=1, yass_alpha=0.01)),
    "gmres_restart4": ("be_small", 150, 2e-6, 2, 0, dict(linear_solver=1, krylov_dim=4)),
    "gmres_no_precond": ("be_small", 150, 2e-6, 2, 0, dict(linear_solver=1, krylov_precond=0)),
    "gmres_gauss_seidel": ("be_small", 150, 2e-6, 2, 0, dict(linear_solver=1, krylov_precond=2)),
    "gmres_gauss_seidel_cv": ("be_small", 150, 2e-6, 2, 1, dict(linear_solver=1, krylov_precond=2)),
    "gmres_jacobi_reactor": ("be_small", 150, 2e-6, 2, 2, dict(linear_solver=1)),
    "gmres_gauss_seidel_reactor": ("be_small", 150, 2e-6, 2, 2, dict(linear_solver=1, krylov_precond=2)),
    "hot_states": ("ros2_1m", 150, 1e-7, 5, 0, {}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_yass_matches_oracle(mechs, case):
    gm, om = mechs
    cfg, nc, dt, n_steps, energy, kw = CASES[case]
    T, p, Y = sample_config(cfg, om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    opt = IntegratorOptions(energy=energy, **kw)
    with np.errstate(all="ignore"):
        ref = oracle.integrate_yass(om, y0, dt, n_steps, opt=opt)
    tol, stable, kalt = 1e-8, None, None
    if kw.get("linear_solver") == 1:
        spread, stable, kalt = _sensitivity(om, y0, dt, n_steps, opt, ref)
        tol = max(1e-8, 10.0 * spread)
        assert stable.mean() >= 0.9
    print(f"[gpu] {om.ns} species, YASS {case}", flush=True)
    got, st, cnt = _run(gm, y0, dt, n_steps, energy=energy, **kw)
    err = _check(om, ref, got, st, cnt, stable, kalt)
    n_cmp = nc if stable is None else int(stable.sum())
    print(f"[gpu] YASS {case}: {ref['rejected'].sum()} rejections, {ref['krylov'].sum()} Krylov iterations, "
          f"{n_cmp} of {nc} cells compared, max rel err {err:.2e} (bar {tol:.1e})", flush=True)
    assert err <= tol


def test_yass_h_min_failure_and_budget(mechs):
    gm, om = mechs
    T, p, Y = sample_config("be_small", om.ns, 20)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    for kw in (dict(yass_alpha=1e-300, h_min=1e-9), dict(yass_alpha=1e-300, h_min=0.0, max_steps=3)):
        ref = oracle.integrate_yass(om, y0, 1e-6, 1, opt=IntegratorOptions(**kw))
        got, st, cnt = _run(gm, y0, 1e-6, 1, **kw)
        np.testing.assert_array_equal(st, ref["status"])
        np.testing.assert_array_equal(cnt[1], ref["rejected"])
        assert np.all(cnt[0] == 0) and np.array_equal(got, y0)
    assert np.all(st == oracle.CELL_MAX_STEPS)


def test_yass_argument_errors(mechs):
    from paper_2510_10005_amd import CHEM_PLAIN, CHEM_YASS, Tape, default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    y = torch.ones((om.n, 8), dtype=torch.float64, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(ChemError, match="persistent form"):
        gm.chem_integrate(8, 8, y, None, default_options(method=CHEM_YASS, dt=1e-8, form=CHEM_PLAIN), None, st, None)
    with pytest.raises(ChemError, match="no adjoint tape"):
        gm.chem_integrate(8, 8, y, None, default_options(method=CHEM_YASS, dt=1e-8), Tape(gm, 8, 2), st, None)
    for kw, msg in ((dict(yass_alpha=0.0), "yass_alpha"), (dict(linear_solver=7), "linear_solver"),
                    (dict(krylov_precond=5), "krylov_precond"), (dict(krylov_max_iter=0), "krylov_max_iter")):
        with pytest.raises(ChemError, match=msg):
            gm.chem_integrate(8, 8, y, None, default_options(method=CHEM_YASS, dt=1e-8, **kw), None, st, None)


@pytest.mark.parametrize("solver", [0, 1])
def test_yass_fullsize_sampled_cells_autotuned(solver):
    """The 1024-cell workload over its 2e-5 s at the paper's YASS step (200 steps of 1e-7 s),
    autotuned persistent launch; 32 seeded cells against the oracle."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_YASS, default_options
    gm, om = gpu_mechanism("h2like_10_27")
    cfg = STATE_CONFIGS["be_small"]
    n = cfg.n_cells
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    opts = default_options(method=CHEM_YASS, dt=2e-5, n_steps=200, form=CHEM_PERSISTENT, linear_solver=solver)
    yd = dev_soa(y0, n)
    gm.chem_autotune(n, n, yd, None, opts)
    print(f"[gpu] YASS (solver {solver}) autotuned launch {gm.chem_get_launch(CHEM_YASS, CHEM_PERSISTENT)}",
          flush=True)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, n), dtype=torch.int32, device="cuda")
    gm.chem_integrate(n, n, yd, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    idx = np.random.default_rng(5004).choice(n, size=32, replace=False)
    opt = IntegratorOptions(linear_solver=solver)
    ref = oracle.integrate_yass(om, y0[idx], 2e-5, 200, opt=opt)
    tol, stable, kalt = 1e-8, None, None
    if solver == 1:
        spread, stable, kalt = _sensitivity(om, y0[idx], 2e-5, 200, opt, ref)
        tol = max(1e-8, 10.0 * spread)
        assert stable.mean() >= 0.9
    got = yd[:, idx].cpu().numpy().T
    err = _check(om, ref, got, st.cpu().numpy()[idx], cnt.cpu().numpy()[:, idx], stable, kalt)
    print(f"[gpu] full-size YASS (solver {solver}): max rel err {err:.2e} (bar {tol:.1e})", flush=True)
    assert err <= tol
