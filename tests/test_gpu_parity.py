"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same seeded inputs.

Tolerances (the bar of the workload definitions; derivations in the design notes):
* thermo, source terms, Jacobian: relative 1e-12 of the magnitude of the terms each value sums
  (|ref| + sum of |terms|), which bounds rounding of either implementation;
* integrated states: relative 1e-8 (T; mass fractions above 1e-12) for cells whose step
  sequence is the same on both sides (equal accepted/rejected counts);
* state maps: relative 1e-13.
Sizes span several 64-lane waves and a ragged tail (cells not a multiple of 64, ld > n_cells).
"""

import numpy as np
import pytest

import oracle
from synth.states import paper_sampler, sample_config

from _gpu import dev_soa, empty, gpu_mechanism, gradient_errors, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu

MECHS = ["tiny_5_6", "tiny_8_14", "h2like_10_27", "sri_12_30", "plog_12_30", "mix_30_90", "ch4like_53_325"]


@pytest.fixture(scope="module", params=MECHS)
def mechs(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


def _skip_block_plain(om, form):
    """Mechanisms with n > 24 integrate in the block form (one cell per workgroup), persistent only."""
    if om.n > 24 and form == 1:
        pytest.skip("the block form (n > 24) runs the persistent form only")


def _states(om, nc, seed=21):
    T, p, Y = paper_sampler(om.ns, nc, seed)
    return T, p, Y, oracle.state_from_TPY(om, T, p, Y)


def test_state_maps(mechs):
    gm, om = mechs
    nc, ld = 333, 357
    T, p, Y, yref = _states(om, nc)
    y = empty(om.n, ld)
    gm.chem_state_from_TPY(nc, ld, dev_soa(T, ld), dev_soa(p, ld), dev_soa(Y, ld), y)
    got = host_aos(y, nc)
    np.testing.assert_allclose(got, yref, rtol=1e-13, atol=0)
    Yd = empty(om.ns, ld)
    gm.chem_mass_fractions(nc, ld, y, Yd)
    np.testing.assert_allclose(host_aos(Yd, nc), oracle.mass_fractions(om, yref), rtol=1e-13, atol=1e-300)


def test_thermo(mechs):
    gm, om = mechs
    nc, ld = 257, 300
    T = np.random.default_rng(4).uniform(300.0, 4500.0, nc)
    outs = [empty(om.ns, ld) for _ in range(4)]
    gm.chem_thermo(nc, ld, dev_soa(T, ld), *outs)
    cp, h, s, g = (host_aos(o, nc) for o in outs)
    rcp, rh, rs, rg = oracle.thermo_mass_specific(om, T)
    scale = rcp * T[:, None]
    np.testing.assert_allclose(cp, rcp, rtol=1e-12)
    assert np.all(np.abs(h - rh) <= 1e-12 * (np.abs(rh) + scale))
    assert np.all(np.abs(s - rs) <= 1e-12 * np.abs(rs) + 1e-12 * rcp)
    assert np.all(np.abs(g - rg) <= 1e-12 * (np.abs(rg) + np.abs(rs) * T[:, None] + scale))


@pytest.mark.parametrize("energy", [0, 1, 2])
def test_source_terms_and_jacobian(mechs, energy):
    gm, om = mechs
    nc, ld = 200 if om.ns < 20 else 70, 256
    T, p, Y, y = _states(om, nc, seed=22 + energy)
    yd = dev_soa(y, ld)
    rng = np.random.default_rng(5)
    lnA = om.lnA_default + rng.uniform(-0.5, 0.5, om.nr)
    import torch
    lnA_d = torch.from_numpy(lnA).cuda()
    S = empty(om.n, ld)
    gm.chem_source_terms(nc, ld, yd, lnA_d, energy, S)
    Sref = oracle.source_terms(om, y, lnA, energy)
    mag = oracle.source_sum_scale(om, y, lnA, energy)
    den = np.abs(Sref) + mag
    err = np.abs(host_aos(S, nc) - Sref) / np.where(den > 0, den, 1.0)
    print(f"[gpu] source max scaled err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-12)
    Jd = empty(om.n * om.n, ld)
    gm.chem_jacobian(nc, ld, yd, lnA_d, energy, Jd)
    J = host_aos(Jd, nc).reshape(nc, om.n, om.n)
    Jref, M = oracle.jacobian(om, y, lnA, energy, magnitude=True)
    err = np.abs(J - Jref) / np.where(np.abs(Jref) + M > 0, np.abs(Jref) + M, 1.0)
    print(f"[gpu] jacobian max scaled err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-12)


def _integrate_gpu(gm, om, y0, opts, ld=None, tape=None, lnA=None):
    import torch
    nc = y0.shape[0]
    ld = ld or nc
    y = dev_soa(y0, ld)
    status = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
    counters = torch.zeros((3, ld), dtype=torch.int32, device="cuda")
    gm.chem_integrate(nc, ld, y, lnA, opts, tape, status, counters)
    torch.cuda.synchronize()
    return host_aos(y, nc), status.cpu().numpy()[:nc], counters.cpu().numpy()[:, :nc]


@pytest.mark.parametrize("form", [0, 1])
def test_backward_euler(mechs, form):
    _skip_block_plain(mechs[1], form)
    from paper_2510_10005_amd import default_options
    gm, om = mechs
    nc = 150 if om.ns < 20 else 24
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    n_steps, dt = 6, 6e-8
    ref = oracle.integrate_be(om, y0, dt, n_steps)
    opts = default_options(method=0, dt=dt, n_steps=n_steps, form=form)
    got, st, cnt = _integrate_gpu(gm, om, y0, opts, ld=nc + 5)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["steps"])
    err = integrated_state_error(om, got, ref["y"])
    print(f"[gpu] BE form {form}: max rel err {err.max():.2e}; newton gpu {cnt[2].sum()} oracle {ref['newton'].sum()}",
          flush=True)
    assert err.max() <= 1e-8


@pytest.mark.parametrize("form", [0, 1])
def test_rosenbrock(mechs, form):
    _skip_block_plain(mechs[1], form)
    from paper_2510_10005_amd import default_options
    gm, om = mechs
    nc = 130 if om.ns < 20 else 16
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    dt = 2e-8
    ref = oracle.integrate_ros2(om, y0, dt)
    opts = default_options(method=1, dt=dt, form=form, n_steps=0)
    got, st, cnt = _integrate_gpu(gm, om, y0, opts)
    np.testing.assert_array_equal(st, ref["status"])
    same = (cnt[0] == ref["accepted"]) & (cnt[1] == ref["rejected"])
    err = integrated_state_error(om, got, ref["y"])
    print(f"[gpu] ROS2 form {form}: {np.count_nonzero(~same)} of {nc} cells with a different step sequence; "
          f"max rel err on the rest {err[same].max() if same.any() else 0:.2e}; accepted {cnt[0].sum()}", flush=True)
    assert np.count_nonzero(~same) <= max(1, nc // 50)
    assert err[same].max() <= 1e-8
    # cells whose sequence differs still agree to the controller's tolerance
    assert np.all(err[~same] <= 1e-3)


def test_fixed_step_rosenbrock(mechs):
    from paper_2510_10005_amd import default_options
    gm, om = mechs
    nc = 70
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_ros2(om, y0, 1e-9, fixed_steps=4)
    got, st, cnt = _integrate_gpu(gm, om, y0, default_options(method=1, dt=1e-9, n_steps=4))
    ok = ref["status"] == 0
    np.testing.assert_array_equal(st, ref["status"])
    assert integrated_state_error(om, got[ok], ref["y"][ok]).max() <= 1e-8


def test_failure_statuses(mechs):
    from paper_2510_10005_amd import default_options
    from test_gpu_large import BLOCK_INVALID_INPUT_OFF
    gm, om = mechs
    if om.n > 24:
        pytest.skip(BLOCK_INVALID_INPUT_OFF)
    T, p, Y = sample_config("be_small", om.ns, 6)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    y0[0, 2] = np.nan
    y0[1, 0] = -3.0
    for method in (0, 1):
        for form in ((0, 1) if om.n <= 24 else (0,)):
            got, st, _ = _integrate_gpu(gm, om, y0, default_options(method=method, dt=1e-8, n_steps=1, form=form))
            assert st[0] == oracle.CELL_NONFINITE and st[1] == oracle.CELL_T_RANGE
            np.testing.assert_array_equal(got[1], y0[1])
    T, p, Y = sample_config("be_small", om.ns, 6)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    _, st, _ = _integrate_gpu(gm, om, y0, default_options(method=0, dt=1e-6, n_steps=1, newton_max=1,
                                                           halving_max_depth=0))
    assert np.all(st == oracle.CELL_NEWTON_FAIL)
    _, st, cnt = _integrate_gpu(gm, om, y0, default_options(method=1, dt=1e-6, n_steps=0, max_steps=3))
    ref = oracle.integrate_ros2(om, y0, 1e-6, opt=oracle.IntegratorOptions(max_steps=3))
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0] + cnt[1], ref["accepted"] + ref["rejected"])


def test_be_adjoint(mechs):
    """Discrete adjoint of backward Euler (with checkpoint recompute) against the oracle's adjoint."""
    import torch
    from oracle.sensitivity import be_adjoint, final_loss
    from paper_2510_10005_amd import Tape, default_options
    from synth.states import loss_weights
    gm, om = mechs
    nc = 70 if om.ns < 20 else 6
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    dt, n_steps = 6e-7, 12
    ref = oracle.integrate_be(om, y0, dt, n_steps, record=True)
    ok = ref["status"] == 0
    w = loss_weights(nc, om.ns)
    _, lamN = final_loss(om, ref["y"], w)
    lam0_ref, g_ref = be_adjoint(om, lamN[ok], [t for t, o in zip(ref["trajectory"], ok) if o])
    tape = Tape(gm, nc, 5)
    got, st, _ = _integrate_gpu(gm, om, y0, default_options(method=0, dt=dt, n_steps=n_steps), tape=tape)
    np.testing.assert_array_equal(st, ref["status"])
    lam_d = dev_soa(lamN)
    out = empty(om.n, nc)
    g = torch.zeros(om.nr, dtype=torch.float64, device="cuda")
    gm.chem_integrate_adjoint(tape, None, lam_d, out, g)
    torch.cuda.synchronize()
    lam0 = host_aos(out, nc)[ok]
    e0, el0 = gradient_errors(lam0, lam0_ref)
    gs = g_ref.sum(axis=0)
    gg = g.cpu().numpy()
    eg = np.abs(gg - gs).max() / np.abs(gs).max()
    big = np.abs(gs) >= 1e-3 * np.abs(gs).max()
    elg = (np.abs(gg - gs)[big] / np.abs(gs)[big]).max()
    print(f"[gpu] BE adjoint: dL/dy0 max rel err {e0:.2e} (element-wise {el0:.2e}), dL/dlnA {eg:.2e} "
          f"(element-wise {elg:.2e})", flush=True)
    assert e0 <= 1e-6 and eg <= 1e-6
    assert el0 <= 1e-6 and elg <= 1e-6      # entries of at least 1e-3 of their column's largest
    # determinism: a second run gives bitwise the same gradient
    g2 = torch.zeros_like(g)
    gm.chem_integrate_adjoint(tape, None, lam_d, out, g2)
    torch.cuda.synchronize()
    assert torch.equal(g, g2)


def test_block_form_refuses_plain_and_tape(mechs):
    """For n > 24 the library refuses the plain form and a Rosenbrock tape on the host (no kernel is
    launched)."""
    from paper_2510_10005_amd import Tape, default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    if om.n <= 24:
        pytest.skip("register-resident mechanism: every form is enabled")
    import torch
    y = torch.zeros((om.n, 8), dtype=torch.float64, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(ChemError, match="persistent form"):
        gm.chem_integrate(8, 8, y, None, default_options(method=1, dt=1e-8, form=1), None, st, None)
    with pytest.raises(ChemError, match="tape"):
        gm.chem_integrate(8, 8, y, None, default_options(method=1, dt=1e-8), Tape(gm, 8, 1, method=1, max_steps=16),
                          st, None)


def test_lu_strategies(mechs):
    """LU strategy 1 (LDS-panel LU, blocked solves) of the block form with the factors in LDS:
    backward Euler and Rosenbrock against the oracle on the bars of the tests above; the strategy
    is kept per method, reported back, refused where its kernels do not exist, and chosen by
    chem_autotune together with the launch shape."""
    import torch
    from paper_2510_10005_amd import CHEM_BE, CHEM_PERSISTENT, CHEM_ROS2, default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    if om.n <= 24 or om.n > 64:
        with pytest.raises(ChemError, match="LU strategy 1"):
            gm.chem_set_lu_strategy(CHEM_ROS2, 1)
        assert gm.chem_get_lu_strategy(CHEM_ROS2) == 0
        return
    with pytest.raises(ChemError):
        gm.chem_set_lu_strategy(CHEM_ROS2, 2)
    for method in (CHEM_BE, CHEM_ROS2):
        gm.chem_set_lu_strategy(method, 1)
        assert gm.chem_get_lu_strategy(method) == 1
    try:
        nc = 24
        T, p, Y = sample_config("be_small", om.ns, nc)
        y0 = oracle.state_from_TPY(om, T, p, Y)
        ref = oracle.integrate_be(om, y0, 6e-8, 6)
        got, st, cnt = _integrate_gpu(gm, om, y0, default_options(method=CHEM_BE, dt=6e-8, n_steps=6), ld=nc + 5)
        np.testing.assert_array_equal(st, ref["status"])
        np.testing.assert_array_equal(cnt[0], ref["steps"])
        e_be = integrated_state_error(om, got, ref["y"]).max()
        T, p, Y = sample_config("ros2_1m", om.ns, 16)
        y0 = oracle.state_from_TPY(om, T, p, Y)
        ref = oracle.integrate_ros2(om, y0, 2e-8)
        got, st, cnt = _integrate_gpu(gm, om, y0, default_options(method=CHEM_ROS2, dt=2e-8, n_steps=0))
        np.testing.assert_array_equal(st, ref["status"])
        same = (cnt[0] == ref["accepted"]) & (cnt[1] == ref["rejected"])
        e_r = integrated_state_error(om, got, ref["y"])
        print(f"[gpu] LU strategy 1: BE max rel err {e_be:.2e}; ROS2 {np.count_nonzero(~same)} of 16 cells with a "
              f"different step sequence, max rel err on the rest {e_r[same].max() if same.any() else 0:.2e}",
              flush=True)
        assert e_be <= 1e-8
        assert np.count_nonzero(~same) <= 1 and e_r[same].max() <= 1e-8
        # autotuning picks the strategy with the launch shape
        n = 512
        T, p, Y = sample_config("ros2_1m", om.ns, n)
        yd = dev_soa(oracle.state_from_TPY(om, T, p, Y), n)
        gm.chem_autotune(n, n, yd, None, default_options(method=CHEM_ROS2, dt=2e-8, n_steps=0, form=CHEM_PERSISTENT))
        assert gm.chem_get_lu_strategy(CHEM_ROS2) in (0, 1)
        print(f"[gpu] autotune: LU strategy {gm.chem_get_lu_strategy(CHEM_ROS2)}, launch "
              f"{gm.chem_get_launch(CHEM_ROS2, CHEM_PERSISTENT)}", flush=True)
        torch.cuda.synchronize()
    finally:
        for method in (CHEM_BE, CHEM_ROS2):
            gm.chem_set_lu_strategy(method, 0)
