"""GPU: the single-range polynomial cp thermo (Section 2.1, degree n_p = 7, refitted from the
10-species mechanism's NASA-7 data by the package's refit utility) against the oracle evaluating the
same mechanism file: thermo (cp, h, s, g) within 1e-12 of the summed term magnitudes of the
polynomials, source terms and Jacobian within 1e-12 of theirs, backward-Euler and Rosenbrock
integration with the oracle's step counts and states within 1e-8.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.mechanism import R
from synth.states import sample_config

from _gpu import KERNEL_CACHE, dev_soa, empty, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mechs():
    import __graft_entry__
    from paper_2510_10005_amd import Mechanism
    path = __graft_entry__.refit_mechanism_file()
    print("[gpu] loading the degree-7 refit of h2like_10_27", flush=True)
    return Mechanism(path, KERNEL_CACHE), oracle.load_mechanism(path)


def _poly_mag(om, T):
    """Term-wise size of the cp/R, h/RT and s/R polynomials (their rounding scale)."""
    out = []
    for i in range(om.ns):
        a, h0, s0 = om.poly[i]
        k = np.arange(len(a))
        cp = (np.abs(a)[None, :] * T[:, None] ** k[None, :]).sum(axis=1)
        h = (np.abs(a / (k + 1))[None, :] * T[:, None] ** k[None, :]).sum(axis=1) + abs(h0) / T
        s = abs(a[0]) * np.abs(np.log(T)) + (np.abs(a[1:] / k[1:])[None, :] * T[:, None] ** k[None, 1:]).sum(axis=1) \
            + abs(s0)
        out.append((cp, h, s))
    return out


def test_refit_thermo(mechs):
    gm, om = mechs
    nc, ld = 300, 320
    T = np.linspace(300.0, 3000.0, nc)
    Td = torch.from_numpy(np.concatenate([T, np.full(ld - nc, 1000.0)])).cuda()
    cp, h, s, g = (empty(om.ns, ld) for _ in range(4))
    gm.chem_thermo(nc, ld, Td, cp, h, s, g)
    torch.cuda.synchronize()
    cpR, hRT, sR, gRT, _ = oracle.nasa7_molar(om, T)
    RW = R / om.W
    mags = _poly_mag(om, T)
    worst = 0.0
    for i in range(om.ns):
        mcp, mh, ms = mags[i]
        worst = max(worst, np.max(np.abs(host_aos(cp, nc)[:, i] - cpR[:, i] * RW[i]) / (mcp * RW[i])))
        worst = max(worst, np.max(np.abs(host_aos(h, nc)[:, i] - hRT[:, i] * RW[i] * T) / (mh * RW[i] * T)))
        worst = max(worst, np.max(np.abs(host_aos(s, nc)[:, i] - sR[:, i] * RW[i]) / (ms * RW[i])))
        worst = max(worst, np.max(np.abs(host_aos(g, nc)[:, i] - gRT[:, i] * RW[i] * T) / ((mh + ms) * RW[i] * T)))
    print(f"[gpu] refit thermo max scaled err {worst:.2e}", flush=True)
    assert worst <= 1e-12


@pytest.mark.parametrize("energy", [0, 1])
def test_refit_source_and_jacobian(mechs, energy):
    gm, om = mechs
    nc, ld = 200, 256
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y = oracle.state_from_TPY(om, T, p, Y)
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
    print(f"[gpu] refit source max scaled err {err.max():.2e}, Jacobian {errJ.max():.2e}", flush=True)
    assert err.max() <= 1e-12 and errJ.max() <= 1e-12


@pytest.mark.parametrize("method", ["be", "ros2"])
def test_refit_integration(mechs, method):
    from paper_2510_10005_amd import CHEM_BE, CHEM_PERSISTENT, CHEM_ROS2, default_options
    gm, om = mechs
    nc = 96
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
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
    same = cnt[2 if method == "be" else 0] == ref["newton" if method == "be" else "accepted"]
    assert same.mean() >= 0.97
    err = integrated_state_error(om, host_aos(y, nc), ref["y"])
    print(f"[gpu] refit {method}: {same.sum()} of {nc} cells with the oracle's counts, max rel err "
          f"{err[same].max():.2e}", flush=True)
    assert err[same].max() <= 1e-8
