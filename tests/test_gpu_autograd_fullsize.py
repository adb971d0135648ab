"""GPU: the autograd Function against the oracle adjoint and finite differences, and full-size
sampled parity of the benchmark workloads in the benchmark's launch configuration.

* ChemIntegrate (BE forward + discrete adjoint) vs the oracle's discrete adjoint composed with
  its loss and init-map pull-backs: relative 1e-6 on dL/dlnA, dL/dT0, dL/dY0; plus central
  differences (h = 1e-6) of the GPU forward on sampled ln A_j (the adjoint workload's check); with
  the density held (Appendix B) and in the constant-pressure reactor mode.
* 1,048,576-cell Rosenbrock workload (persistent, autotuned launch): sampled cells vs the oracle
  one by one, relative 1e-8 where the step sequences agree.
* 1024-cell backward-Euler workload (200 x 1e-7 s): sampled cells vs the oracle, relative 1e-8.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.integrate import IntegratorOptions
from oracle.sensitivity import be_adjoint, final_loss, init_map_vjp
from synth.states import STATE_CONFIGS, loss_weights, sample_config, sample_states

from _gpu import gpu_mechanism, integrated_state_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    return gpu_mechanism("h2like_10_27")


@pytest.mark.parametrize("energy", [0, 2])
def test_autograd_matches_oracle_adjoint_and_fd(small, energy):
    from paper_2510_10005_amd.autograd import chem_integrate
    gm, om = small
    nc, dt, nst = 48, 4e-7, 20
    T, p, Y = sample_config("be_small", om.ns, nc)
    w = loss_weights(nc, om.ns)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T0 = d(T).requires_grad_(True)
    Y0 = d(Y.T).requires_grad_(True)
    lnA = d(om.lnA_default).requires_grad_(True)
    print(f"[gpu] autograd, energy mode {energy}", flush=True)
    TN, YN, st = chem_integrate(T0, Y0, lnA, gm, d(p), dt, nst, checkpoint_every=6, energy=energy)
    L = TN.sum() + (d(w.T) * YN).sum()
    L.backward()
    assert torch.all(st == 0)
    # oracle: forward with trajectory, loss pull-back, adjoint, init-map pull-back
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_be(om, y0, dt, nst, record=True, opt=IntegratorOptions(energy=energy))
    _, lamN = final_loss(om, ref["y"], w)
    lam0, g = be_adjoint(om, lamN, ref["trajectory"], energy=energy)
    dT_ref, dY_ref = init_map_vjp(om, T, p, Y, lam0)
    g_ref = g.sum(axis=0)

    def rel(a, b):
        return np.abs(a - b).max() / np.abs(b).max()
    eA = rel(lnA.grad.cpu().numpy(), g_ref)
    eT = rel(T0.grad.cpu().numpy(), dT_ref)
    eY = rel(Y0.grad.cpu().numpy().T, dY_ref)
    print(f"[gpu] autograd vs oracle adjoint: lnA {eA:.2e}, T0 {eT:.2e}, Y0 {eY:.2e}", flush=True)
    assert eA < 1e-6 and eT < 1e-6 and eY < 1e-6
    # central differences of the GPU forward on sampled reactions
    h = 1e-6
    rng = np.random.default_rng(4000)
    for j in rng.choice(om.nr, size=6, replace=False):
        vals = []
        for s in (+1, -1):
            la = lnA.detach().clone()
            la[j] += s * h
            with torch.no_grad():
                TN2, YN2, _ = chem_integrate(T0.detach(), Y0.detach(), la, gm, d(p), dt, nst, energy=energy)
                vals.append(float(TN2.sum() + (d(w.T) * YN2).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        noise = 4e-16 * abs(float(L)) / h
        assert abs(fd - float(lnA.grad[j])) <= 1e-6 * abs(float(lnA.grad[j])) + noise, (j, fd, float(lnA.grad[j]))


def test_fullsize_rosenbrock_sampled_cells(small):
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, default_options
    gm, om = small
    cfg = STATE_CONFIGS["ros2_1m"]
    n = cfg.n_cells
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y = torch.empty((om.n, n), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(n, n, d(T), d(p), d(Y.T), y)
    opts = default_options(method=CHEM_ROS2, dt=1e-6, n_steps=0, form=CHEM_PERSISTENT)
    gm.chem_autotune(1 << 17, n, y, None, opts)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, n), dtype=torch.int32, device="cuda")
    gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    idx = np.random.default_rng(5000).choice(n, size=6, replace=False)
    got = y[:, idx].cpu().numpy().T
    ref = oracle.integrate_ros2(om, oracle.state_from_TPY(om, T[idx], p[idx], Y[idx]), 1e-6)
    c = cnt[:, idx].cpu().numpy()
    same = (c[0] == ref["accepted"]) & (c[1] == ref["rejected"])
    err = integrated_state_error(om, got, ref["y"])
    print(f"[gpu] full-size ROS2: {same.sum()} of {len(idx)} sampled cells with identical step sequences, "
          f"max rel err {err[same].max() if same.any() else 0:.2e}; all cells status 0: {bool((st == 0).all())}")
    assert np.all(st[idx].cpu().numpy() == ref["status"])
    assert same.sum() >= len(idx) - 1
    assert err[same].max() <= 1e-8
    assert np.all(err <= 1e-3)


def test_fullsize_backward_euler_sampled_cells(small):
    from paper_2510_10005_amd import CHEM_BE, default_options
    gm, om = small
    cfg = STATE_CONFIGS["be_small"]
    n = cfg.n_cells
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y = torch.empty((om.n, n), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(n, n, d(T), d(p), d(Y.T), y)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    gm.chem_integrate(n, n, y, None, default_options(method=CHEM_BE, dt=2e-5, n_steps=200), None, st, None)
    torch.cuda.synchronize()
    idx = np.random.default_rng(5001).choice(n, size=32, replace=False)
    ref = oracle.integrate_be(om, oracle.state_from_TPY(om, T[idx], p[idx], Y[idx]), 2e-5, 200)
    err = integrated_state_error(om, y[:, idx].cpu().numpy().T, ref["y"])
    print(f"[gpu] full-size BE: max rel err {err.max():.2e}")
    assert np.all(st[idx].cpu().numpy() == ref["status"])
    assert err.max() <= 1e-8


@pytest.mark.parametrize("mech_name,cfg_name", [("h2like_10_27", "ros2_1m"), ("ch4like_53_325", "ros2_methane")])
def test_fullsize_source_and_jacobian_sampled_cells(mech_name, cfg_name):
    """Source terms and Jacobian over the benchmark's full state sets (1,048,576 cells of the
    10-species mechanism, 262,144 of the 53-species one), 12 sampled cells against the oracle
    at the 1e-12 scaled tolerance of the parity tests."""
    gm, om = gpu_mechanism(mech_name)
    cfg = STATE_CONFIGS[cfg_name]
    n = cfg.n_cells
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y = torch.empty((om.n, n), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(n, n, d(T), d(p), d(Y.T), y)
    S = torch.empty_like(y)
    gm.chem_source_terms(n, n, y, None, 0, S)
    idx = np.sort(np.random.default_rng(5002).choice(n, size=12, replace=False))
    idx_d = torch.from_numpy(idx).cuda()
    ys = y[:, idx_d].cpu().numpy().T
    Ss = S[:, idx_d].cpu().numpy().T
    del S
    J = torch.empty((om.n * om.n, n), dtype=torch.float64, device="cuda")
    gm.chem_jacobian(n, n, y, None, 0, J)
    Js = J[:, idx_d].cpu().numpy().T.reshape(-1, om.n, om.n)
    del J
    Sref = oracle.source_terms(om, ys)
    mag = oracle.source_sum_scale(om, ys)
    den = np.abs(Sref) + mag
    es = np.abs(Ss - Sref) / np.where(den > 0, den, 1.0)
    Jref, M = oracle.jacobian(om, ys, magnitude=True)
    ej = np.abs(Js - Jref) / np.where(np.abs(Jref) + M > 0, np.abs(Jref) + M, 1.0)
    print(f"[gpu] full-size {mech_name}: source {es.max():.2e}, jacobian {ej.max():.2e} (scaled)", flush=True)
    assert es.max() <= 1e-12 and ej.max() <= 1e-12
