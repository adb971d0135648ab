"""GPU parity of the constant-pressure reactor form (energy CHEM_CONST_P_REACTOR) against the oracle.

* the block form's backward Euler and Rosenbrock (n > 24, both LU strategies where they exist):
  states within 1e-8 relative, equal step counts, the bar of the other integrator tests;
* the block-form source-term and Jacobian kernels of the 150-species mechanism: relative 1e-12 of
  the magnitude of the terms each value sums (the API kernels of the smaller mechanisms are covered
  by the energy parametrisation of the parity suite);
* the register-resident form (n <= 24) runs the reactor mode with its full-system build (every
  species in the solved system): backward Euler (persistent and plain), Rosenbrock (persistent and
  plain), SDIRK-2, SDIRK-4 and YASS with LU against the oracle on the same bar, and the regular
  build keeps running the other modes in the same process;
* the backward-Euler discrete adjoint in the reactor mode (dilatation terms in the transposed
  Jacobian and in the ln A contraction), block form and the register form's full-system build,
  against the oracle's adjoint, 1e-6 element-wise;
* the host refuses the reactor form for the other adjoint tapes and unknown energy modes before any
  kernel runs.
"""

import numpy as np
import pytest

import oracle
from oracle.integrate import IntegratorOptions
from synth.states import paper_sampler, sample_config

from _gpu import dev_soa, empty, gpu_mechanism, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu

REACTOR = 2
_ROS2_REF = {}   # oracle runs shared by the two LU strategies


@pytest.fixture(scope="module", params=["mix_30_90", "ch4like_53_325"])
def block_mech(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


def _integrate_gpu(gm, y0, opts, ld):
    import torch
    nc = y0.shape[0]
    y = dev_soa(y0, ld)
    status = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
    counters = torch.zeros((3, ld), dtype=torch.int32, device="cuda")
    gm.chem_integrate(nc, ld, y, None, opts, None, status, counters)
    torch.cuda.synchronize()
    return host_aos(y, nc), status.cpu().numpy()[:nc], counters.cpu().numpy()[:, :nc]


@pytest.mark.parametrize("lus", [0, 1])
def test_reactor_backward_euler(block_mech, lus):
    from paper_2510_10005_amd import CHEM_BE, default_options
    gm, om = block_mech
    nc = 40
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_be(om, y0, 6e-8, 6, opt=IntegratorOptions(energy=REACTOR))
    gm.chem_set_lu_strategy(CHEM_BE, lus)
    try:
        print(f"[gpu] reactor BE n={om.n} lus={lus}", flush=True)
        got, st, cnt = _integrate_gpu(gm, y0, default_options(method=CHEM_BE, dt=6e-8, n_steps=6, energy=REACTOR),
                                      nc + 5)
    finally:
        gm.chem_set_lu_strategy(CHEM_BE, 0)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["steps"])
    err = integrated_state_error(om, got, ref["y"])
    print(f"[gpu] reactor BE max rel err {err.max():.2e}; newton gpu {cnt[2].sum()} oracle {ref['newton'].sum()}",
          flush=True)
    assert err.max() <= 1e-8
    # the density-holding form gives another answer (the dilatation terms are not negligible here)
    held = oracle.integrate_be(om, y0, 6e-8, 6)
    assert integrated_state_error(om, got, held["y"]).max() > 1e-6


@pytest.mark.parametrize("lus", [0, 1])
def test_reactor_rosenbrock(block_mech, lus):
    from paper_2510_10005_amd import CHEM_ROS2, default_options
    gm, om = block_mech
    nc, dt = 16, 3e-9
    T, p, Y = sample_config("ros2_methane", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    if om.n not in _ROS2_REF:
        _ROS2_REF[om.n] = oracle.integrate_ros2(om, y0, dt, opt=IntegratorOptions(energy=REACTOR))
    ref = _ROS2_REF[om.n]
    gm.chem_set_lu_strategy(CHEM_ROS2, lus)
    try:
        print(f"[gpu] reactor ROS2 n={om.n} lus={lus}", flush=True)
        got, st, cnt = _integrate_gpu(gm, y0, default_options(method=CHEM_ROS2, dt=dt, energy=REACTOR), nc + 3)
    finally:
        gm.chem_set_lu_strategy(CHEM_ROS2, 0)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["accepted"])
    np.testing.assert_array_equal(cnt[1], ref["rejected"])
    err = integrated_state_error(om, got, ref["y"])
    print(f"[gpu] reactor ROS2 max rel err {err.max():.2e}; accepted {cnt[0].sum()}", flush=True)
    assert err.max() <= 1e-8


def _register_ref(om, y0, method, dt, n_steps):
    opt = IntegratorOptions(energy=REACTOR)
    if method == "be":
        return oracle.integrate_be(om, y0, dt, n_steps, opt=opt)
    if method == "ros2":
        return oracle.integrate_ros2(om, y0, dt, opt=opt)
    if method == "sdirk2":
        return oracle.integrate_sdirk2(om, y0, dt, n_steps, opt=opt)
    if method == "sdirk4":
        return oracle.integrate_sdirk4(om, y0, dt, n_steps, opt=opt)
    return oracle.integrate_yass(om, y0, dt, n_steps, opt=opt)


_REGISTER_REF = {}   # oracle runs shared by the persistent and plain forms
REGISTER_CASES = {
    # name: (method, form, dt, n_steps)
    "be": ("be", 0, 2e-6, 4),
    "be_plain": ("be", 1, 2e-6, 4),
    "ros2": ("ros2", 0, 2e-7, 0),
    "ros2_plain": ("ros2", 1, 2e-7, 0),
    "sdirk2": ("sdirk2", 0, 2e-6, 4),
    "sdirk4": ("sdirk4", 0, 2e-6, 4),
    "yass_lu": ("yass", 0, 2e-6, 2),
}


@pytest.mark.parametrize("name", ["tiny_8_14", "h2like_10_27"])
@pytest.mark.parametrize("case", list(REGISTER_CASES))
def test_reactor_register_form(name, case):
    import paper_2510_10005_amd as P
    from paper_2510_10005_amd import default_options
    gm, om = gpu_mechanism(name)
    method, form, dt, n_steps = REGISTER_CASES[case]
    nc = 130
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    key = (name, method, dt, n_steps)
    if key not in _REGISTER_REF:
        with np.errstate(all="ignore"):
            _REGISTER_REF[key] = _register_ref(om, y0, method, dt, n_steps)
    ref = _REGISTER_REF[key]
    code = {"be": P.CHEM_BE, "ros2": P.CHEM_ROS2, "sdirk2": P.CHEM_SDIRK2, "sdirk4": P.CHEM_SDIRK4,
            "yass": P.CHEM_YASS}[method]
    print(f"[gpu] reactor {name} {case}", flush=True)
    got, st, cnt = _integrate_gpu(gm, y0, default_options(method=code, dt=dt, n_steps=n_steps, form=form,
                                                          energy=REACTOR), nc + 3)
    np.testing.assert_array_equal(st, ref["status"])
    if "steps" in ref:
        np.testing.assert_array_equal(cnt[0], ref["steps"])
    else:
        np.testing.assert_array_equal(cnt[0], ref["accepted"])
        np.testing.assert_array_equal(cnt[1], ref["rejected"])
    ok = ref["status"] == 0
    err = integrated_state_error(om, got[ok], ref["y"][ok])
    print(f"[gpu] reactor {name} {case}: {ok.sum()} cells, max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 1e-8
    # the inert collider's concentration changes with the density (the reduced system holds it)
    inert = 1 + np.nonzero(om.inert)[0]
    assert np.abs(got[ok][:, inert] / y0[ok][:, inert] - 1.0).max() > 1e-6
    # the regular build still serves the density-holding mode in the same process
    if case == "be":
        held = oracle.integrate_be(om, y0, dt, n_steps)
        g0, s0, c0 = _integrate_gpu(gm, y0, default_options(method=code, dt=dt, n_steps=n_steps), nc + 3)
        np.testing.assert_array_equal(s0, held["status"])
        assert integrated_state_error(om, g0[s0 == 0], held["y"][s0 == 0]).max() <= 1e-8
        assert np.array_equal(g0[:, inert], y0[:, inert])


def test_reactor_failure_statuses_register_form():
    """Per-cell statuses in the reactor mode (full-system build): non-finite and T <= 0 input cells
    (both forms, backward Euler and Rosenbrock), Newton failure without halving, the attempt budget."""
    import paper_2510_10005_amd as P
    from paper_2510_10005_amd import default_options
    gm, om = gpu_mechanism("h2like_10_27")
    T, p, Y = sample_config("be_small", om.ns, 6)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    bad = y0.copy()
    bad[0, 2] = np.nan
    bad[1, 0] = -3.0
    for method in (P.CHEM_BE, P.CHEM_ROS2):
        for form in (P.CHEM_PERSISTENT, P.CHEM_PLAIN):
            got, st, _ = _integrate_gpu(gm, bad, default_options(method=method, dt=1e-8, n_steps=1, form=form,
                                                                 energy=REACTOR), 9)
            assert st[0] == oracle.CELL_NONFINITE and st[1] == oracle.CELL_T_RANGE
            np.testing.assert_array_equal(got[1], bad[1])
            assert np.all(st[2:] == 0)
    _, st, _ = _integrate_gpu(gm, y0, default_options(method=P.CHEM_BE, dt=1e-6, n_steps=1, newton_max=1,
                                                      halving_max_depth=0, energy=REACTOR), 9)
    assert np.all(st == oracle.CELL_NEWTON_FAIL)
    _, st, cnt = _integrate_gpu(gm, y0, default_options(method=P.CHEM_ROS2, dt=1e-6, max_steps=3, energy=REACTOR), 9)
    with np.errstate(all="ignore"):
        ref = oracle.integrate_ros2(om, y0, 1e-6, opt=IntegratorOptions(max_steps=3, energy=REACTOR))
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0] + cnt[1], ref["accepted"] + ref["rejected"])


def test_reactor_rosenbrock_launch_shape_larger_system():
    """The 12-species mechanism's reduced system (12 components) parks its U factor in 159,744 B of
    LDS at 256 threads per block; the full-system build (13) would need 186,368 B.  A launch shape
    set for the regular build is narrowed for the reactor mode instead of failing, in both forms."""
    import paper_2510_10005_amd as P
    from paper_2510_10005_amd import default_options
    gm, om = gpu_mechanism("sri_12_30")
    nc = 96
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    with np.errstate(all="ignore"):
        ref = oracle.integrate_ros2(om, y0, 1e-7, opt=IntegratorOptions(energy=REACTOR))
    for form in (P.CHEM_PERSISTENT, P.CHEM_PLAIN):
        gm.chem_set_launch(P.CHEM_ROS2, form, 256, 0)
        try:
            print(f"[gpu] reactor ROS2 12 species, form {form}, block 256 requested", flush=True)
            got, st, cnt = _integrate_gpu(gm, y0, default_options(method=P.CHEM_ROS2, dt=1e-7, form=form,
                                                                  energy=REACTOR), nc + 3)
        finally:
            gm.chem_set_launch(P.CHEM_ROS2, form, 0, 0)
        np.testing.assert_array_equal(st, ref["status"])
        np.testing.assert_array_equal(cnt[0], ref["accepted"])
        assert integrated_state_error(om, got, ref["y"]).max() <= 1e-8


def test_reactor_autotune_register_form():
    """chem_autotune in the reactor mode times the full-system build's kernels (its occupancy and
    LDS limits) and leaves a launch shape that integrates correctly."""
    import paper_2510_10005_amd as P
    from paper_2510_10005_amd import default_options
    gm, om = gpu_mechanism("mid_14_40")
    nc = 2000
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    opts = default_options(method=P.CHEM_ROS2, dt=1e-7, energy=REACTOR)
    gm.chem_autotune(nc, nc, dev_soa(y0, nc), None, opts)
    print(f"[gpu] reactor autotuned launch {gm.chem_get_launch(P.CHEM_ROS2, P.CHEM_PERSISTENT)}", flush=True)
    idx = np.arange(0, nc, 16)
    with np.errstate(all="ignore"):
        ref = oracle.integrate_ros2(om, y0[idx], 1e-7, opt=IntegratorOptions(energy=REACTOR))
    try:
        got, st, cnt = _integrate_gpu(gm, y0, opts, nc)
    finally:
        gm.chem_set_launch(P.CHEM_ROS2, P.CHEM_PERSISTENT, 0, 0)
    np.testing.assert_array_equal(st[idx], ref["status"])
    np.testing.assert_array_equal(cnt[0][idx], ref["accepted"])
    assert integrated_state_error(om, got[idx], ref["y"]).max() <= 1e-8


def test_reactor_be_adjoint_block_form(block_mech):
    _reactor_be_adjoint(*block_mech, 8)


@pytest.mark.parametrize("name", ["tiny_8_14", "h2like_10_27"])
def test_reactor_be_adjoint_register_form(name):
    """The register form's backward-Euler adjoint in the reactor mode: the full-system build's
    adjoint kernel (replays on the full system, dilatation terms in the ln A contraction)."""
    _reactor_be_adjoint(*gpu_mechanism(name), 70)


def _reactor_be_adjoint(gm, om, nc):
    import torch
    from oracle.sensitivity import be_adjoint, final_loss
    from paper_2510_10005_amd import CHEM_BE, Tape, default_options
    from synth.states import loss_weights
    from _gpu import gradient_errors
    dt, n_steps, K = 6e-8, 6, 4
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_be(om, y0, dt, n_steps, record=True, opt=IntegratorOptions(energy=REACTOR))
    assert np.all(ref["status"] == 0)
    _, lamN = final_loss(om, ref["y"], loss_weights(nc, om.ns))
    lam0_ref, g_ref = be_adjoint(om, lamN, ref["trajectory"], energy=REACTOR)
    tape = Tape(gm, nc, K)
    print(f"[gpu] reactor BE adjoint n={om.n}, {nc} cells", flush=True)
    got, st, _ = _integrate_gpu_tape(gm, y0, default_options(method=CHEM_BE, dt=dt, n_steps=n_steps, energy=REACTOR),
                                     nc, tape)
    np.testing.assert_array_equal(st, ref["status"])
    assert integrated_state_error(om, got, ref["y"]).max() <= 1e-8
    out = empty(om.n, nc)
    g = torch.zeros(om.nr, dtype=torch.float64, device="cuda")
    gm.chem_integrate_adjoint(tape, None, dev_soa(lamN), out, g)
    torch.cuda.synchronize()
    e0, el0 = gradient_errors(host_aos(out, nc), lam0_ref)
    eg, elg = gradient_errors(g.cpu().numpy()[None, :], g_ref.sum(axis=0)[None, :])
    print(f"[gpu] reactor BE adjoint: dL/dy0 {e0:.2e} (element-wise {el0:.2e}), dL/dlnA {eg:.2e} "
          f"(element-wise {elg:.2e})", flush=True)
    assert max(e0, el0, eg, elg) <= 1e-6
    # the density-holding adjoint differs (the dilatation terms matter here)
    lam0_held, _ = be_adjoint(om, lamN, ref["trajectory"])
    assert gradient_errors(host_aos(out, nc), lam0_held)[0] > 1e-6


def _integrate_gpu_tape(gm, y0, opts, ld, tape):
    import torch
    nc = y0.shape[0]
    y = dev_soa(y0, ld)
    status = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
    counters = torch.zeros((3, ld), dtype=torch.int32, device="cuda")
    gm.chem_integrate(nc, ld, y, None, opts, tape, status, counters)
    torch.cuda.synchronize()
    return host_aos(y, nc), status.cpu().numpy()[:nc], counters.cpu().numpy()[:, :nc]


def test_reactor_api_kernels_150_species():
    import torch
    gm, om = gpu_mechanism("large_150_1000")
    nc, ld = 37, 40
    T, p, Y = paper_sampler(om.ns, nc, 23)
    y = oracle.state_from_TPY(om, T, p, Y)
    yd = dev_soa(y, ld)
    lnA = om.lnA_default + np.random.default_rng(6).uniform(-0.5, 0.5, om.nr)
    lnA_d = torch.from_numpy(lnA).cuda()
    print("[gpu] reactor API kernels, 150 species", flush=True)
    S = empty(om.n, ld)
    gm.chem_source_terms(nc, ld, yd, lnA_d, REACTOR, S)
    Sref = oracle.source_terms(om, y, lnA, REACTOR)
    den = np.abs(Sref) + oracle.source_sum_scale(om, y, lnA, REACTOR)
    err = np.abs(host_aos(S, nc) - Sref) / np.where(den > 0, den, 1.0)
    print(f"[gpu] source max scaled err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-12)
    Jd = empty(om.n * om.n, ld)
    gm.chem_jacobian(nc, ld, yd, lnA_d, REACTOR, Jd)
    J = host_aos(Jd, nc).reshape(nc, om.n, om.n)
    Jref, M = oracle.jacobian(om, y, lnA, REACTOR, magnitude=True)
    err = np.abs(J - Jref) / np.where(np.abs(Jref) + M > 0, np.abs(Jref) + M, 1.0)
    print(f"[gpu] jacobian max scaled err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-12)


def test_reactor_refusals():
    import torch
    from paper_2510_10005_amd import CHEM_BE, CHEM_ROS2, Tape, default_options
    from paper_2510_10005_amd._binding import ChemError
    small, om_s = gpu_mechanism("h2like_10_27")
    y = torch.zeros((om_s.n, 8), dtype=torch.float64, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(ChemError, match="tape"):
        small.chem_integrate(8, 8, y, None, default_options(method=CHEM_ROS2, dt=1e-8, energy=REACTOR),
                             Tape(small, 8, 1, method=CHEM_ROS2, max_steps=16), st, None)
    big, om_b = gpu_mechanism("mix_30_90")
    yb = torch.zeros((om_b.n, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ChemError, match="tape"):
        big.chem_integrate(8, 8, yb, None, default_options(method=CHEM_ROS2, dt=1e-8, energy=REACTOR),
                           Tape(big, 8, 1), st, None)
    with pytest.raises(ChemError, match="energy"):
        big.chem_integrate(8, 8, yb, None, default_options(method=CHEM_BE, dt=1e-8, n_steps=1, energy=3), None, st,
                           None)
