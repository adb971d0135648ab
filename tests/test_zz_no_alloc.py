"""GPU: the allocation-free integration entry point against chem_integrate.

chem_integrate_noalloc takes every workspace from the library's per-device scratch array.  Two
calls in a row, the second on fewer cells, must reproduce chem_integrate bit for bit (same
kernels, same step sequences), for the adaptive Rosenbrock method with the probe/resume schedule
and for backward Euler, with and without a caller-supplied counters array, and for the
Rosenbrock method in the constant-pressure reactor mode (the full-system build, which the entry
point refuses to load and uses once chem_integrate has loaded it).  Sizes above the array's limit
are refused on the host.
"""

import pytest

from synth.states import sample_config

from _gpu import dev_soa, gpu_mechanism

pytestmark = pytest.mark.gpu


def _states(om, nc):
    import oracle
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    return oracle.state_from_TPY(om, T, p, Y)


def _pair(gm, y0, ld, opts, with_counters):
    """(state, status, counters) from chem_integrate and from chem_integrate_noalloc."""
    import torch
    nc = y0.shape[0]
    out = []
    for noalloc in (False, True):
        y = dev_soa(y0, ld)
        st = torch.full((ld,), -7, dtype=torch.int32, device="cuda")
        cnt = torch.zeros((3, ld), dtype=torch.int32, device="cuda") if with_counters else None
        if noalloc:
            gm.chem_integrate_noalloc(nc, ld, y, None, opts, st, cnt)
        else:
            gm.chem_integrate(nc, ld, y, None, opts, None, st, cnt)
        torch.cuda.synchronize()
        out.append((y[:, :nc].clone(), st[:nc].clone(), None if cnt is None else cnt[:, :nc].clone()))
    return out


@pytest.mark.parametrize("method", [1, 0])
def test_noalloc_matches_integrate_two_calls(method):
    import torch
    from paper_2510_10005_amd import default_options
    gm, om = gpu_mechanism("h2like_10_27")
    opts = (default_options(method=1, dt=2e-7, n_steps=0, probe_attempts=16) if method == 1
            else default_options(method=0, dt=1e-7, n_steps=20))
    for nc, ld, with_counters in ((3000, 3011, True), (1100, 1100, False)):
        print(f"[gpu] noalloc method {method}: {nc} cells, ld {ld}, counters {with_counters}", flush=True)
        y0 = _states(om, nc)
        (ya, sa, ca), (yb, sb, cb) = _pair(gm, y0, ld, opts, with_counters)
        assert torch.equal(ya, yb)
        assert torch.equal(sa, sb)
        if with_counters:
            assert torch.equal(ca, cb)
        assert int((sa == 0).sum().item()) == nc


def test_noalloc_refuses_oversized_calls():
    import torch
    from paper_2510_10005_amd import default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = gpu_mechanism("h2like_10_27")
    y = torch.zeros((om.n, 8), dtype=torch.float64, device="cuda")
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(ChemError, match="at most"):
        gm.chem_integrate_noalloc((1 << 20) + 1, (1 << 20) + 1, y, None, default_options(method=1, dt=1e-8), st, None)
    with pytest.raises(ChemError, match="persistent"):
        gm.chem_integrate_noalloc(8, 8, y, None, default_options(method=1, dt=1e-8, form=1), st, None)


def test_noalloc_reactor_mode_after_full_system_load():
    import torch
    from paper_2510_10005_amd import CHEM_CONST_P_REACTOR, default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = gpu_mechanism("h2like_10_27")
    opts = default_options(method=1, dt=2e-7, n_steps=0, probe_attempts=16, energy=CHEM_CONST_P_REACTOR)
    y = dev_soa(_states(om, 8), 8)
    st = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(ChemError, match="full-system build"):
        gm.chem_integrate_noalloc(8, 8, y, None, opts, st, None)
    for nc, ld, with_counters in ((3000, 3011, True), (1100, 1100, False)):
        print(f"[gpu] noalloc reactor mode: {nc} cells, ld {ld}, counters {with_counters}", flush=True)
        y0 = _states(om, nc)
        (ya, sa, ca), (yb, sb, cb) = _pair(gm, y0, ld, opts, with_counters)
        assert torch.equal(ya, yb)
        assert torch.equal(sa, sb)
        if with_counters:
            assert torch.equal(ca, cb)
        assert int((sa == 0).sum().item()) == nc
        # the density change reaches the inert collider (the full-system build ran)
        inert = 1 + torch.nonzero(torch.as_tensor(om.inert)).flatten().to("cuda")
        assert not torch.equal(ya[inert], dev_soa(y0, ld)[inert, :nc])
