"""GPU: discrete adjoint of the two-stage Rosenbrock integration against the oracle's reverse sweep.

The forward run records its accepted steps on a Rosenbrock tape (persistent form); the adjoint
replays each checkpoint segment and walks it backwards.  The oracle differentiates its own
recorded step sequence (oracle.sensitivity.ros2_adjoint), so the GPU's accepted-step counts must
equal the oracle's first.  Checked: adaptive steps and fixed steps (where the second-derivative
terms change the gradient by percents), both energy modes, segments that end mid-way
(checkpoint_every not dividing the step count), the probe/resume schedule during recording
(bitwise equal to a single launch), a tape capacity below some cells' step counts (those cells
stop with status 3 and get a zero adjoint), and bitwise-reproducible gradients.
Tolerance 1e-6 relative (dL/dy0 per component against the largest |value| of that component
over the cells, and element by element on the entries of at least 1e-3 of it; dL/dlnA against
its largest |value|).
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.sensitivity import final_loss, ros2_adjoint
from synth.states import loss_weights, sample_config

from _gpu import dev_soa, empty, gpu_mechanism, gradient_errors, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu

MECHS = ["tiny_5_6", "tiny_8_14", "h2like_10_27", "sri_12_30", "plog_12_30"]


@pytest.fixture(scope="module", params=MECHS)
def mechs(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


def _forward(gm, om, y0, opts, tape, ld):
    nc = y0.shape[0]
    y = dev_soa(y0, ld)
    st = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, ld), dtype=torch.int32, device="cuda")
    gm.chem_integrate(nc, ld, y, None, opts, tape, st, cnt)
    torch.cuda.synchronize()
    return host_aos(y, nc), st.cpu().numpy()[:nc], cnt.cpu().numpy()[:, :nc]


def _adjoint(gm, om, tape, lamN, ld):
    nc = lamN.shape[0]
    out = empty(om.n, ld)
    g = torch.zeros(om.nr, dtype=torch.float64, device="cuda")
    gm.chem_integrate_adjoint(tape, None, dev_soa(lamN, ld), out, g)
    torch.cuda.synchronize()
    return host_aos(out, nc), g.cpu().numpy()


def _errors(lam0, g, lam0_ref, g_ref):
    scale = np.abs(lam0_ref).max(axis=0, keepdims=True)
    e0 = np.abs(lam0 - lam0_ref) / np.where(scale > 0, scale, 1.0)
    gs = g_ref.sum(axis=0)
    eg = np.abs(g - gs) / max(np.abs(gs).max(), 1e-300)
    return e0.max(), eg.max()


CASES = {
    # name: (dt, fixed steps, checkpoint_every, energy, probe_attempts)
    "adaptive": (1e-9, 0, 4, 0, 0),
    "adaptive_cv": (1e-9, 0, 3, 1, 0),
    "fixed": (1e-7, 5, 2, 0, 0),
    "adaptive_probe": (1e-9, 0, 4, 0, 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_ros2_adjoint_matches_oracle(mechs, case):
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, Tape, default_options
    gm, om = mechs
    dt, fixed, K, energy, budget = CASES[case]
    nc = 24
    ld = nc + 3
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_ros2(om, y0, dt, opt=oracle.IntegratorOptions(energy=energy), record=True,
                                fixed_steps=fixed)
    if not np.all(ref["status"] == 0):
        # a fixed step too long for a cell of this mechanism (the oracle's own run fails there):
        # compare on the cells it integrates
        keep = ref["status"] == 0
        assert keep.mean() >= 0.9
        y0 = y0[keep]
        nc = int(keep.sum())
        ld = nc + 3
        ref = oracle.integrate_ros2(om, y0, dt, opt=oracle.IntegratorOptions(energy=energy), record=True,
                                    fixed_steps=fixed)
        assert np.all(ref["status"] == 0)
    w = loss_weights(nc, om.ns)
    _, lamN = final_loss(om, ref["y"], w)
    lam0_ref, g_ref = ros2_adjoint(om, lamN, y0, ref["history"], energy=energy)
    print(f"[gpu] {om.ns} species, case {case}: forward with tape", flush=True)
    tape = Tape(gm, nc, K, method=CHEM_ROS2, max_steps=int(ref["accepted"].max()) + 1)
    opts = default_options(method=CHEM_ROS2, dt=dt, n_steps=fixed, energy=energy, form=CHEM_PERSISTENT,
                           probe_attempts=budget)
    got, st, cnt = _forward(gm, om, y0, opts, tape, ld)
    bad = (st != ref["status"]) | (cnt[0] != ref["accepted"])
    assert not bad.any(), (f"status {st[bad]} vs {ref['status'][bad]}, accepted {cnt[0][bad]} vs "
                           f"{ref['accepted'][bad]}, rejected {cnt[1][bad]} vs {ref['rejected'][bad]}")
    assert integrated_state_error(om, got, ref["y"]).max() <= 1e-8
    print(f"[gpu] {om.ns} species, case {case}: adjoint", flush=True)
    lam0, g = _adjoint(gm, om, tape, lamN, ld)
    e0, eg = _errors(lam0, g, lam0_ref, g_ref)
    el0 = gradient_errors(lam0, lam0_ref)[1]
    print(f"[gpu] ROS2 adjoint {case}: dL/dy0 max rel err {e0:.2e} (element-wise on entries >= 1e-3 of the column "
          f"maximum {el0:.2e}), dL/dlnA max rel err {eg:.2e}", flush=True)
    assert e0 <= 1e-6 and eg <= 1e-6 and el0 <= 1e-6
    lam0b, g2 = _adjoint(gm, om, tape, lamN, ld)
    assert np.array_equal(g, g2) and np.array_equal(lam0, lam0b)


def test_probe_resume_recording_is_bitwise_identical(mechs):
    """Recording with a small probe budget (cells parked and resumed) gives the same tape."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, Tape, default_options
    gm, om = mechs
    nc = 300
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    lamN = final_loss(om, y0, loss_weights(nc, om.ns))[1]
    res = []
    for budget in (0, 2):
        print(f"[gpu] {om.ns} species: recording with probe budget {budget}", flush=True)
        tape = Tape(gm, nc, 3, method=CHEM_ROS2, max_steps=64)
        opts = default_options(method=CHEM_ROS2, dt=2e-9, form=CHEM_PERSISTENT, probe_attempts=budget)
        got, st, cnt = _forward(gm, om, y0, opts, tape, nc)
        lam0, g = _adjoint(gm, om, tape, lamN, nc)
        res.append((got, st, cnt, lam0, g))
    a, b = res
    assert (a[2][0] + a[2][1] > 2).any()      # some cells were parked
    for x, y in zip(a, b):
        assert np.array_equal(np.nan_to_num(x, nan=7.0), np.nan_to_num(y, nan=7.0))


def test_tape_capacity(mechs):
    """Cells needing more accepted steps than the tape holds stop with status 3, adjoint zero."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, Tape, default_options
    gm, om = mechs
    nc = 40
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    dt = 1e-9 if om.ns >= 8 else 1e-8     # a spread of accepted-step counts over the cells
    ref = oracle.integrate_ros2(om, y0, dt, record=True)
    acc = ref["accepted"]
    assert acc.min() < acc.max()
    cap = max(1, int(acc.min() + acc.max()) // 2)
    over = acc > cap
    tape = Tape(gm, nc, 2, method=CHEM_ROS2, max_steps=cap)
    print(f"[gpu] {om.ns} species: tape capacity {cap}", flush=True)
    opts = default_options(method=CHEM_ROS2, dt=dt, form=CHEM_PERSISTENT)
    _, st, cnt = _forward(gm, om, y0, opts, tape, nc)
    np.testing.assert_array_equal(st, np.where(over, 3, 0))
    np.testing.assert_array_equal(cnt[0], np.minimum(ref["accepted"], cap))
    lamN = final_loss(om, ref["y"], loss_weights(nc, om.ns))[1]
    lam0, g = _adjoint(gm, om, tape, lamN, nc)
    assert np.all(lam0[over] == 0.0)
    ok = ~over
    lam0_ref, g_ref = ros2_adjoint(om, lamN[ok], y0[ok], [h for h, o in zip(ref["history"], ok) if o])
    e0, eg = _errors(lam0[ok], g, lam0_ref, g_ref)
    assert e0 <= 1e-6 and eg <= 1e-6


def test_tape_argument_errors(mechs):
    from paper_2510_10005_amd import CHEM_BE, CHEM_PLAIN, CHEM_ROS2, Tape, default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    y = torch.ones((om.n, 8), dtype=torch.float64, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    tape = Tape(gm, 8, 2, method=CHEM_ROS2, max_steps=10)
    with pytest.raises(ChemError, match="another method"):
        gm.chem_integrate(8, 8, y, None, default_options(method=CHEM_BE, dt=1e-8, n_steps=2), tape, st, None)
    with pytest.raises(ChemError, match="persistent form"):
        gm.chem_integrate(8, 8, y, None, default_options(method=CHEM_ROS2, dt=1e-8, form=CHEM_PLAIN), tape, st, None)
    with pytest.raises(ChemError, match="no recorded"):
        out = torch.empty_like(y)
        gm.chem_integrate_adjoint(tape, None, y, out, torch.zeros(om.nr, dtype=torch.float64, device="cuda"))
    with pytest.raises(ChemError, match="max_steps"):
        Tape(gm, 8, 2, method=CHEM_ROS2, max_steps=0)


def test_autograd_rosenbrock_matches_oracle():
    """torch.autograd through (T0, Y0, lnA) -> (T_N, Y_N) with the Rosenbrock method."""
    from oracle.sensitivity import init_map_vjp
    from paper_2510_10005_amd import CHEM_ROS2
    from paper_2510_10005_amd.autograd import chem_integrate
    gm, om = gpu_mechanism("h2like_10_27")
    nc, dt, fixed = 24, 1e-7, 5
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    w = loss_weights(nc, om.ns)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T0 = d(T).requires_grad_(True)
    Y0 = d(Y.T).requires_grad_(True)
    lnA = d(om.lnA_default).requires_grad_(True)
    print("[gpu] autograd Rosenbrock: forward + backward", flush=True)
    TN, YN, st = chem_integrate(T0, Y0, lnA, gm, d(p), dt, fixed, checkpoint_every=2, method=CHEM_ROS2, max_steps=8)
    L = TN.sum() + (d(w.T) * YN).sum()
    L.backward()
    assert torch.all(st == 0)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_ros2(om, y0, dt, record=True, fixed_steps=fixed)
    _, lamN = final_loss(om, ref["y"], w)
    lam0, g = ros2_adjoint(om, lamN, y0, ref["history"])
    dT_ref, dY_ref = init_map_vjp(om, T, p, Y, lam0)

    def rel(a, b):
        return np.abs(a - b).max() / np.abs(b).max()
    eA = rel(lnA.grad.cpu().numpy(), g.sum(axis=0))
    eT = rel(T0.grad.cpu().numpy(), dT_ref)
    eY = rel(Y0.grad.cpu().numpy().T, dY_ref)
    print(f"[gpu] autograd Rosenbrock vs oracle adjoint: lnA {eA:.2e}, T0 {eT:.2e}, Y0 {eY:.2e}", flush=True)
    assert eA < 1e-6 and eT < 1e-6 and eY < 1e-6
