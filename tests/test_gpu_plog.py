"""GPU: P-log rates (Section 2.2) on the 12-species P-log mechanism (one cell per lane) and on the
30-species mechanism with P-log and SRI reactions (one cell per wavefront) at pressures from 3e3 to 3e6 Pa,
so that every interval of the pressure tables and both clamps are exercised (the other GPU tests
run it at one atmosphere only).  Source terms and Jacobian within 1e-12 of the summed term
magnitudes, both energy modes; backward-Euler and Rosenbrock integration with the oracle's step
counts and states within 1e-8.
"""

import numpy as np
import pytest
import torch

import oracle
from synth.states import sample_config

from _gpu import dev_soa, empty, gpu_mechanism, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mechs():
    print("[gpu] loading plog_12_30", flush=True)
    return gpu_mechanism("plog_12_30")


@pytest.fixture(scope="module", params=["plog_12_30", "mix_30_90"])
def any_form(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


def _states(om, n, seed):
    T, _, Y = sample_config("ros2_1m", om.ns, n)
    p = np.geomspace(3e3, 3e6, n)
    np.random.default_rng(seed).shuffle(p)
    return oracle.state_from_TPY(om, T, p, Y)


@pytest.mark.parametrize("energy", [0, 1])
def test_plog_source_and_jacobian(any_form, energy):
    gm, om = any_form
    nc, ld = 240, 256
    y = _states(om, nc, 3 + energy)
    yd = dev_soa(y, ld)
    S = empty(om.n, ld)
    gm.chem_source_terms(nc, ld, yd, None, energy, S)
    Sref = oracle.source_terms(om, y, None, energy)
    den = np.abs(Sref) + oracle.source_sum_scale(om, y, None, energy)
    err = np.abs(host_aos(S, nc) - Sref) / np.where(den > 0, den, 1.0)
    Jd = empty(om.n * om.n, ld)
    gm.chem_jacobian(nc, ld, yd, None, energy, Jd)
    J = host_aos(Jd, nc).reshape(nc, om.n, om.n)
    Jref, M = oracle.jacobian(om, y, None, energy, magnitude=True)
    errJ = np.abs(J - Jref) / np.where(np.abs(Jref) + M > 0, np.abs(Jref) + M, 1.0)
    print(f"[gpu] P-log source max scaled err {err.max():.2e}, Jacobian {errJ.max():.2e}", flush=True)
    assert err.max() <= 1e-12 and errJ.max() <= 1e-12


@pytest.mark.parametrize("method", ["be", "ros2"])
def test_plog_integration(mechs, method):
    from paper_2510_10005_amd import CHEM_BE, CHEM_PERSISTENT, CHEM_ROS2, default_options
    gm, om = mechs
    nc = 96
    y0 = _states(om, nc, 11)
    if method == "be":
        ref = oracle.integrate_be(om, y0, 1e-7, 4)
        opts = default_options(method=CHEM_BE, dt=1e-7, n_steps=4, form=CHEM_PERSISTENT)
    else:
        ref = oracle.integrate_ros2(om, y0, 1e-8)
        opts = default_options(method=CHEM_ROS2, dt=1e-8, form=CHEM_PERSISTENT)
    y = dev_soa(y0, nc)
    st = torch.full((nc,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, nc), dtype=torch.int32, device="cuda")
    gm.chem_integrate(nc, nc, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    st, cnt = st.cpu().numpy(), cnt.cpu().numpy()
    np.testing.assert_array_equal(st, ref["status"])
    key = "newton" if method == "be" else "accepted"
    same = cnt[2 if method == "be" else 0] == ref[key]
    assert same.mean() >= 0.97
    err = integrated_state_error(om, host_aos(y, nc), ref["y"])
    print(f"[gpu] P-log {method}: {same.sum()} of {nc} cells with the oracle's counts, max rel err "
          f"{err[same].max():.2e}", flush=True)
    assert err[same].max() <= 1e-8
