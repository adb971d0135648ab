"""GPU: the 53-species mechanism's integration workloads in the benchmark's launch configurations,
checked against oracle references stored by committed scripts that call only oracle/
(tests/golden/make_ros2_methane_samples.py, tests/golden/make_adjoint_methane_samples.py); the
oracle needs minutes per cell at these horizons, so its results are stored rather than recomputed.

* adaptive Rosenbrock over 1e-5 s on 4,096 cells with the 262,144-cell set's distribution and
  seed (block form, persistent queue with probe/resume, autotuned grid): 8 sampled cells, equal
  step counts and integrated states within 1e-8;
* differentiation workload (16,384 cells, backward Euler 500 x 2e-8 s, checkpoints every 50): the
  forward with tape at full size, then one adjoint whose dL/dy_N is the loss pull-back on 3
  sampled cells and on the first 64 cells (zero elsewhere; the adjoint is linear in it): dL/dy0 of
  the 3 cells against the oracle's discrete adjoint and of the 64 cells against the oracle's
  tangent (forward-sensitivity) reference, dL/dlnA summed over the 67 cells against both, all
  within 1e-6 of each column's largest entry and element by element on the entries of at least
  1e-3 of it;
* the same adjoint on the first 64 cells against central differences (h = 1e-6) of the GPU
  forward on 32 ln A_j sampled with seed 4000.
"""

import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle.sensitivity import final_loss
from synth.states import STATE_CONFIGS, loss_weights, sample_states

from _gpu import gpu_mechanism, gradient_errors, integrated_state_error

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def methane():
    print("[gpu] loading ch4like_53_325", flush=True)
    return gpu_mechanism("ch4like_53_325")


def _device_states(gm, T, p, Y):
    n = T.shape[0]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y = torch.empty((gm.n, n), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(n, n, d(T), d(p), d(Y.T), y)
    return y


def test_methane_rosenbrock_subset_sampled_cells(methane):
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, default_options
    gm, om = methane
    ref = json.load(open(os.path.join(GOLDEN, "ros2_methane_samples.json")))
    n = ref["subset"]
    cfg = STATE_CONFIGS["ros2_methane"]
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)   # = sample_config(.., n)
    y = _device_states(gm, T, p, Y)
    opts = default_options(method=CHEM_ROS2, dt=ref["dt"], n_steps=0, rtol=ref["rtol"], atol=ref["atol"],
                           form=CHEM_PERSISTENT)
    print(f"[gpu] 53-species ROS2: autotune on 1024 cells, then {n} cells over {ref['dt']:g} s", flush=True)
    gm.chem_autotune(1024, n, y.clone(), None, opts)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, n), dtype=torch.int32, device="cuda")
    gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    idx = [r["cell"] for r in ref["cells"]]
    got = y[:, idx].cpu().numpy().T
    c = cnt[:, idx].cpu().numpy()
    yo = np.array([r["y"] for r in ref["cells"]])
    same = (c[0] == [r["accepted"] for r in ref["cells"]]) & (c[1] == [r["rejected"] for r in ref["cells"]])
    err = integrated_state_error(om, got, yo).max(axis=1)
    print(f"[gpu] 53-species ROS2: {int(same.sum())} of {len(idx)} sampled cells with equal step counts, max rel "
          f"err {err.max():.2e}; substeps per cell {int(cnt[0].min())}..{int(cnt[0].max())}", flush=True)
    assert np.all(st.cpu().numpy()[idx] == [r["status"] for r in ref["cells"]])
    assert np.all(same)
    assert err.max() <= 1e-8


def test_methane_adjoint_fullsize_vs_oracle_adjoint_and_tangent(methane):
    from paper_2510_10005_amd import CHEM_BE, Tape, default_options
    gm, om = methane
    ref = json.load(open(os.path.join(GOLDEN, "adjoint_methane_samples.json")))
    N = ref["cells_total"]
    cfg = STATE_CONFIGS["adjoint_methane"]
    T, p, Y = sample_states(om.ns, N, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    y = _device_states(gm, T, p, Y)
    st = torch.empty(N, dtype=torch.int32, device="cuda")
    tape = Tape(gm, N, 50)
    print(f"[gpu] 53-species BE forward with tape ({N} cells, {ref['n_steps']} steps)", flush=True)
    gm.chem_integrate(N, N, y, None, default_options(method=CHEM_BE, dt=ref["dt"], n_steps=ref["n_steps"]),
                      tape, st, None)
    torch.cuda.synchronize()
    stc = st.cpu().numpy()
    yN = y.cpu().numpy().T
    adj = ref["adjoint"]["cells"]
    ia = [a["cell"] for a in adj]
    it = ref["tangent"]["cells"]
    assert all(a["status"] == 0 for a in adj) and np.all(np.array(ref["tangent"]["status"]) == 0)
    assert np.all(stc[ia] == 0) and np.all(stc[it] == 0)
    # the forward states at the sampled cells match the oracle's
    assert integrated_state_error(om, yN[ia], np.array([a["y"] for a in adj])).max() <= 1e-8
    # dL/dy_N: the loss pull-back at the GPU's final states on the 67 cells, zero elsewhere
    w = loss_weights(N, om.ns)
    cells = np.array(sorted(set(ia) | set(it)))
    _, lam_c = final_loss(om, yN[cells], w[cells])
    lam = np.zeros((om.n, N))
    lam[:, cells] = lam_c.T
    lam_d = torch.from_numpy(lam).cuda()
    out = torch.empty_like(lam_d)
    g = torch.zeros(om.nr, dtype=torch.float64, device="cuda")
    print("[gpu] 53-species BE adjoint (sparse dL/dy_N)", flush=True)
    gm.chem_integrate_adjoint(tape, None, lam_d, out, g)
    torch.cuda.synchronize()
    d0 = out.cpu().numpy().T
    gg = g.cpu().numpy()

    e_adj, el_adj = gradient_errors(d0[ia], np.array([a["dLdy0"] for a in adj]))
    e_tan, el_tan = gradient_errors(d0[it], np.array(ref["tangent"]["dLdy0"]))
    g_ref = np.array(ref["adjoint"]["dLdlnA_sum"]) + np.array(ref["tangent"]["dLdlnA_sum"])
    e_g = np.abs(gg - g_ref).max() / np.abs(g_ref).max()
    big = np.abs(g_ref) >= 1e-3 * np.abs(g_ref).max()
    el_g = (np.abs(gg - g_ref)[big] / np.abs(g_ref)[big]).max()
    print(f"[gpu] 53-species adjoint: dL/dy0 vs oracle adjoint {e_adj:.2e} (element-wise {el_adj:.2e}), vs oracle "
          f"tangent {e_tan:.2e} ({el_tan:.2e}); dL/dlnA {e_g:.2e} ({el_g:.2e})", flush=True)
    assert e_adj <= 1e-6 and e_tan <= 1e-6 and e_g <= 1e-6
    # element by element on the entries of at least 1e-3 of their column's (dL/dlnA: vector's) largest
    assert el_adj <= 1e-6 and el_tan <= 1e-6 and el_g <= 1e-6


def test_methane_adjoint_vs_central_differences(methane):
    from paper_2510_10005_amd import CHEM_BE, Tape, default_options
    gm, om = methane
    n, dt, nst, h = 64, 1e-5, 500, 1e-6
    cfg = STATE_CONFIGS["adjoint_methane"]
    # the first 64 cells of the 16,384-cell set (the tangent reference's cells), their loss weights
    T, p, Y = (a[:n] for a in sample_states(om.ns, cfg.n_cells, cfg.seed, cfg.T_range, cfg.alpha, cfg.p))
    y0 = _device_states(gm, T, p, Y)
    w = loss_weights(cfg.n_cells, om.ns)[:n]
    opts = default_options(method=CHEM_BE, dt=dt, n_steps=nst)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, n), dtype=torch.int32, device="cuda")

    def forward(lnA, tape=None):
        y = y0.clone()
        gm.chem_integrate(n, n, y, torch.from_numpy(lnA).cuda(), opts, tape, st, cnt)
        torch.cuda.synchronize()
        assert torch.all(st == 0)
        L, lam = final_loss(om, y.cpu().numpy().T, w)
        return L, lam, cnt[2].cpu().numpy().copy()

    lnA0 = np.array(om.lnA_default, dtype=np.float64)
    tape = Tape(gm, n, 50)
    L0, lamN, _ = forward(lnA0, tape)
    out = torch.empty((om.n, n), dtype=torch.float64, device="cuda")
    g = torch.zeros(om.nr, dtype=torch.float64, device="cuda")
    gm.chem_integrate_adjoint(tape, torch.from_numpy(lnA0).cuda(), torch.from_numpy(np.ascontiguousarray(lamN.T)).cuda(),
                              out, g)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    js = np.random.default_rng(4000).choice(om.nr, size=32, replace=False)
    print(f"[gpu] central differences on 32 ln A_j ({n} cells, {nst} steps)", flush=True)
    worst, same_newton = 0.0, 0
    noise = 4e-16 * abs(L0) / h
    for j in js:
        vals, newt = [], []
        for s in (+1, -1):
            la = lnA0.copy()
            la[j] += s * h
            L, _, nw = forward(la)
            vals.append(L)
            newt.append(nw)
        fd = (vals[0] - vals[1]) / (2 * h)
        if not np.array_equal(newt[0], newt[1]):
            continue      # a different Newton iteration count makes the forward map non-smooth here
        same_newton += 1
        err = abs(fd - g[j]) / (abs(g[j]) + noise / 1e-6)
        worst = max(worst, err)
        assert abs(fd - g[j]) <= 1e-6 * abs(g[j]) + noise, (int(j), fd, float(g[j]))
    print(f"[gpu] central differences: {same_newton} of 32 parameters with equal Newton counts, worst scaled "
          f"error {worst:.2e}", flush=True)
    assert same_newton >= 24
