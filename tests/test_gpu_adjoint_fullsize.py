"""GPU: both discrete adjoints at the benchmark's full sizes and launch configuration, checked on
sampled cells.

The adjoint is linear in dL/dy_N, so the benchmark's 16,384-cell runs are repeated with dL/dy_N
nonzero only on three seeded cells: every other cell then contributes exactly zero, and dL/dy0 of
the sampled cells and the cell-summed dL/dlnA can be compared with the oracle's adjoint of those
cells alone (relative 1e-6).

* backward Euler, 10-species mechanism, 500 x 2e-8 s, checkpoints every 50 (the adjoint workload);
* adaptive Rosenbrock over 1e-6 s on the headline state distribution, checkpoints every 50; the
  three cells are the ones with the fewest accepted steps among 16 seeded candidates (chosen by the
  oracle's forward run), and their GPU step counts must equal the oracle's.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.sensitivity import be_adjoint, final_loss, ros2_adjoint
from synth.states import STATE_CONFIGS, loss_weights, sample_states

from _gpu import gpu_mechanism, gradient_errors

pytestmark = pytest.mark.gpu

N = 16384


@pytest.fixture(scope="module")
def small():
    return gpu_mechanism("h2like_10_27")


def _device_states(gm, T, p, Y):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y = torch.empty((gm.n, N), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(N, N, d(T), d(p), d(Y.T), y)
    return y


def _sparse_adjoint(gm, tape, idx, lam_rows):
    lam = np.zeros((gm.n, N))
    lam[:, idx] = lam_rows.T
    lam_d = torch.from_numpy(lam).cuda()
    out = torch.empty_like(lam_d)
    g = torch.zeros(gm.nr, dtype=torch.float64, device="cuda")
    gm.chem_integrate_adjoint(tape, None, lam_d, out, g)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:, idx].T, g.cpu().numpy()


def _check(lam0, g, lam0_ref, g_ref, label):
    e0, el0 = gradient_errors(lam0, lam0_ref)
    gs = g_ref.sum(axis=0)
    eg = np.abs(g - gs).max() / np.abs(gs).max()
    big = np.abs(gs) >= 1e-3 * np.abs(gs).max()
    elg = (np.abs(g - gs)[big] / np.abs(gs)[big]).max()
    print(f"[gpu] full-size {label} adjoint, sampled cells: dL/dy0 {e0:.2e} (element-wise {el0:.2e}), dL/dlnA "
          f"{eg:.2e} (element-wise {elg:.2e})", flush=True)
    assert e0 <= 1e-6 and eg <= 1e-6
    assert el0 <= 1e-6 and elg <= 1e-6    # entries of at least 1e-3 of their column's largest


def test_fullsize_be_adjoint_sampled_cells(small):
    from paper_2510_10005_amd import CHEM_BE, Tape, default_options
    gm, om = small
    cfg = STATE_CONFIGS["adjoint_methane"]
    T, p, Y = sample_states(om.ns, N, cfg.seed, (1000.0, 1500.0), 1.0, cfg.p)
    idx = np.sort(np.random.default_rng(5003).choice(N, size=3, replace=False))
    y = _device_states(gm, T, p, Y)
    st = torch.empty(N, dtype=torch.int32, device="cuda")
    tape = Tape(gm, N, 50)
    print("[gpu] full-size BE forward with tape (16,384 cells, 500 steps)", flush=True)
    gm.chem_integrate(N, N, y, None, default_options(method=CHEM_BE, dt=1e-5, n_steps=500), tape, st, None)
    torch.cuda.synchronize()
    y0 = oracle.state_from_TPY(om, T[idx], p[idx], Y[idx])
    ref = oracle.integrate_be(om, y0, 1e-5, 500, record=True)
    assert np.all(ref["status"] == 0) and np.all(st.cpu().numpy()[idx] == 0)
    _, lamN = final_loss(om, ref["y"], loss_weights(N, om.ns)[idx])
    lam0_ref, g_ref = be_adjoint(om, lamN, ref["trajectory"])
    lam0, g = _sparse_adjoint(gm, tape, idx, lamN)
    _check(lam0, g, lam0_ref, g_ref, "BE")


def test_fullsize_ros2_adjoint_sampled_cells(small):
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, Tape, default_options
    gm, om = small
    cfg = STATE_CONFIGS["ros2_1m"]
    T, p, Y = sample_states(om.ns, N, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    cand = np.sort(np.random.default_rng(5002).choice(N, size=16, replace=False))
    y0c = oracle.state_from_TPY(om, T[cand], p[cand], Y[cand])
    ref = oracle.integrate_ros2(om, y0c, 1e-6, record=True)
    pick = np.argsort(ref["accepted"], kind="stable")[:3]
    idx = cand[pick]
    y = _device_states(gm, T, p, Y)
    st = torch.empty(N, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, N), dtype=torch.int32, device="cuda")
    tape = Tape(gm, N, 50, method=CHEM_ROS2, max_steps=20000)
    print("[gpu] full-size Rosenbrock forward with tape (16,384 cells, 1e-6 s)", flush=True)
    gm.chem_integrate(N, N, y, None, default_options(method=CHEM_ROS2, dt=1e-6, form=CHEM_PERSISTENT), tape, st, cnt)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()
    np.testing.assert_array_equal(c[0][idx], ref["accepted"][pick])
    np.testing.assert_array_equal(c[1][idx], ref["rejected"][pick])
    assert np.all(st.cpu().numpy()[idx] == 0)
    lamN = np.random.default_rng(3001).standard_normal((3, om.n)) / np.abs(ref["y"][pick])
    lam0_ref, g_ref = ros2_adjoint(om, lamN, y0c[pick], [ref["history"][i] for i in pick])
    lam0, g = _sparse_adjoint(gm, tape, idx, lamN)
    _check(lam0, g, lam0_ref, g_ref, "Rosenbrock")
