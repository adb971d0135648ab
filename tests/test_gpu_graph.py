"""GPU: the persistent split step captured in a HIP graph.

The persistent form of chem_integrate issues two kernels (queue reset, integrator) and no
allocation once its buffers exist, so it can be captured.  Each replay re-integrates the same
initial states; every replay must reproduce the eager call bit for bit (cells are independent and
each lane runs the same instruction sequence), with eager work and synchronisations between the
replays.  Both the register form (10 species) and the block form (53 species, one cell per
workgroup, probe/resume schedule) are captured, and the constant-pressure reactor mode (energy 2:
the register form's full-system build) as well.
"""

import numpy as np
import pytest
import torch

from synth.states import STATE_CONFIGS, sample_states

from _gpu import gpu_mechanism

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mech,method,n,energy", [("h2like_10_27", "ros2", 6000, 0), ("h2like_10_27", "be", 6000, 0),
                                                  ("ch4like_53_325", "ros2", 600, 0), ("ch4like_53_325", "be", 600, 0),
                                                  ("h2like_10_27", "ros2", 6000, 2), ("ch4like_53_325", "be", 600, 2)])
def test_graph_replay_matches_eager(mech, method, n, energy):
    from paper_2510_10005_amd import CHEM_BE, CHEM_PERSISTENT, CHEM_ROS2, default_options
    gm, om = gpu_mechanism(mech)
    cfg = STATE_CONFIGS["ros2_1m"]
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y0 = torch.empty((om.n, n), dtype=torch.float64, device="cuda")
    gm.chem_state_from_TPY(n, n, d(T), d(p), d(Y.T), y0)
    if method == "ros2":
        opts = default_options(method=CHEM_ROS2, dt=1e-6, n_steps=0, form=CHEM_PERSISTENT, energy=energy)
    else:
        opts = default_options(method=CHEM_BE, dt=1e-6, n_steps=20, form=CHEM_PERSISTENT, energy=energy)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, n), dtype=torch.int32, device="cuda")
    # eager reference (also allocates the library's internal buffers before capture)
    y.copy_(y0)
    gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    y_ref, st_ref, cnt_ref = y.clone(), st.clone(), cnt.clone()

    g = torch.cuda.CUDAGraph()
    y.copy_(y0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
    torch.cuda.synchronize()
    src = torch.empty_like(y0)
    for r in range(4):
        y.copy_(y0)
        st.fill_(-1)
        cnt.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), f"replay {r}: states differ"
        assert torch.equal(st, st_ref), f"replay {r}: statuses differ"
        assert torch.equal(cnt, cnt_ref), f"replay {r}: counters differ"
        gm.chem_source_terms(n, n, y0, None, 0, src)     # unrelated eager work between replays
        torch.cuda.synchronize()
    print(f"[gpu] graph replay ({method}): 4 replays identical to eager, "
          f"{int(cnt_ref[0].sum())} accepted substeps", flush=True)
