"""GPU: degenerate sizes and argument errors of the C ABI (10-species mechanism).

* n_cells = 0 is a no-op for every entry point: outputs keep their contents.
* One cell with ld = 1 integrates like the oracle (both methods, both forms).
* Argument errors are reported before any launch: ld < n_cells, negative n_cells.
"""

import numpy as np
import pytest
import torch

import oracle
from synth.states import sample_config

from _gpu import gpu_mechanism, integrated_state_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mech():
    return gpu_mechanism("h2like_10_27")


def _full(shape, v, dtype=torch.float64):
    return torch.full(shape, v, dtype=dtype, device="cuda")


def test_empty_batch_is_a_noop(mech):
    from paper_2510_10005_amd import CHEM_BE, CHEM_PERSISTENT, CHEM_PLAIN, CHEM_ROS2, Tape, default_options
    gm, om = mech
    ld = 4
    y = _full((om.n, ld), 7.0)
    out = _full((om.n, ld), -3.0)
    jac = _full((om.n * om.n, ld), -3.0)
    gm.chem_source_terms(0, ld, y, None, 0, out)
    gm.chem_jacobian(0, ld, y, None, 0, jac)
    outs = [_full((om.ns, ld), -3.0) for _ in range(4)]
    gm.chem_thermo(0, ld, y[0], *outs)
    st = _full((ld,), 5, torch.int32)
    cnt = _full((3, ld), 9, torch.int32)
    for method in (CHEM_BE, CHEM_ROS2):
        for form in (CHEM_PERSISTENT, CHEM_PLAIN):
            gm.chem_integrate(0, ld, y, None, default_options(method=method, dt=1e-8, form=form), None, st, cnt)
    tape = Tape(gm, 0, 1)
    gm.chem_integrate(0, ld, y, None, default_options(method=CHEM_BE, dt=1e-8, n_steps=2), tape, st, cnt)
    torch.cuda.synchronize()
    assert torch.all(out == -3.0) and torch.all(jac == -3.0) and all(torch.all(o == -3.0) for o in outs)
    assert torch.all(y == 7.0) and torch.all(st == 5) and torch.all(cnt == 9)


@pytest.mark.parametrize("method,form", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_single_cell(mech, method, form):
    from paper_2510_10005_amd import default_options
    gm, om = mech
    T, p, Y = sample_config("ros2_1m", om.ns, 1)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    y = torch.from_numpy(np.ascontiguousarray(y0.T)).cuda()
    st = _full((1,), -9, torch.int32)
    cnt = torch.zeros((3, 1), dtype=torch.int32, device="cuda")
    if method == 0:
        opts = default_options(method=0, dt=5e-8, n_steps=5, form=form)
        ref = oracle.integrate_be(om, y0, 5e-8, 5)
    else:
        opts = default_options(method=1, dt=2e-8, n_steps=0, form=form)
        ref = oracle.integrate_ros2(om, y0, 2e-8)
    gm.chem_integrate(1, 1, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    assert int(st[0]) == int(ref["status"][0])
    assert integrated_state_error(om, y.cpu().numpy().T, ref["y"]).max() <= 1e-8


def test_argument_errors(mech):
    from paper_2510_10005_amd import default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mech
    y = _full((om.n, 8), 1.0)
    out = _full((om.n, 8), 0.0)
    st = _full((8,), 0, torch.int32)
    with pytest.raises(ChemError, match="ld must be"):
        gm.chem_source_terms(8, 4, y, None, 0, out)
    with pytest.raises(ChemError, match="n_cells must be"):
        gm.chem_source_terms(-1, 8, y, None, 0, out)
    with pytest.raises(ChemError, match="ld must be"):
        gm.chem_integrate(8, 4, y, None, default_options(method=1, dt=1e-8), None, st, None)
    with pytest.raises(ChemError, match="dt must be"):
        gm.chem_integrate(8, 8, y, None, default_options(method=1, dt=0.0), None, st, None)
    with pytest.raises(ChemError, match="probe_attempts"):
        gm.chem_integrate(8, 8, y, None, default_options(method=1, dt=1e-8, probe_attempts=-1), None, st, None)
