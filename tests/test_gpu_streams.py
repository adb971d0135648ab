"""GPU: calls on one mechanism from two streams, and launch shapes whose LDS does not fit.

* The mechanism's work queue, schedule and continuation buffers are shared by every stream.  Two
  persistent Rosenbrock integrations enqueued back to back on two streams must give bitwise the
  results of the same integrations run one after the other (the library orders the second call
  after the first), and a subset of them must match the oracle at the integrated-state bar.
* The constant-pressure reactor mode runs a second build of a register-resident mechanism; which
  build a call uses is chosen per call.  Two host threads, each on its own stream, one in the
  reactor mode and one holding the density, calling the same mechanism at the same time, must give
  bitwise the results of the same calls made one after the other.
* The Rosenbrock kernels of the register-resident form park the upper LU factor in LDS, one packed
  triangle per lane, so their LDS grows with the block size.  For a 14-species mechanism (13 active
  species) a block of 256 lanes would need more than the device's LDS per block: chem_set_launch refuses it,
  chem_autotune skips it and keeps a working shape, and the integration still matches the oracle.
"""

import numpy as np
import pytest

import oracle
from synth.states import sample_config

from _gpu import dev_soa, gpu_mechanism, host_aos, integrated_state_error

pytestmark = pytest.mark.gpu


def _cells(om, cfg, nc, seed_shift=0):
    T, p, Y = sample_config(cfg, om.ns, nc + seed_shift)
    return oracle.state_from_TPY(om, T[seed_shift:], p[seed_shift:], Y[seed_shift:])


def _run(gm, om, y0, dt, stream=None, energy=0):
    import torch
    from paper_2510_10005_amd import default_options
    nc = y0.shape[0]
    y = dev_soa(y0)
    st = torch.full((nc,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((3, nc), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    opts = default_options(method=1, dt=dt, n_steps=0, energy=energy)
    if stream is None:
        gm.chem_integrate(nc, nc, y, None, opts, None, st, cnt)
    else:
        with torch.cuda.stream(stream):
            gm.chem_integrate(nc, nc, y, None, opts, None, st, cnt)
    return y, st, cnt


def test_two_streams_share_one_mechanism():
    import torch
    gm, om = gpu_mechanism("h2like_10_27")
    yA0 = _cells(om, "ros2_1m", 6000)
    yB0 = _cells(om, "ros2_1m", 1500, seed_shift=7)
    print("[gpu] serial reference runs", flush=True)
    rA, sA_ref, cA_ref = _run(gm, om, yA0, 1e-7)
    rB, sB_ref, cB_ref = _run(gm, om, yB0, 5e-8)
    torch.cuda.synchronize()
    print("[gpu] concurrent runs on two streams", flush=True)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    yA, sA, cA = _run(gm, om, yA0, 1e-7, s1)
    yB, sB, cB = _run(gm, om, yB0, 5e-8, s2)
    torch.cuda.synchronize()
    assert torch.equal(yA, rA) and torch.equal(sA, sA_ref) and torch.equal(cA, cA_ref)
    assert torch.equal(yB, rB) and torch.equal(sB, sB_ref) and torch.equal(cB, cB_ref)
    # and the oracle on a subset of the second batch
    k = 40
    ref = oracle.integrate_ros2(om, yB0[:k], 5e-8)
    got = host_aos(yB, yB0.shape[0])[:k]
    cnt = cB.cpu().numpy()[:, :k]
    same = (cnt[0] == ref["accepted"]) & (cnt[1] == ref["rejected"])
    np.testing.assert_array_equal(sB.cpu().numpy()[:k], ref["status"])
    assert np.count_nonzero(~same) <= 1
    assert integrated_state_error(om, got[same], ref["y"][same]).max() <= 1e-8


def test_two_threads_reactor_and_density_holding_modes():
    import threading
    import torch
    from paper_2510_10005_amd import CHEM_CONST_P_REACTOR
    gm, om = gpu_mechanism("h2like_10_27")
    jobs = [(_cells(om, "ros2_1m", 3000), 1e-7, CHEM_CONST_P_REACTOR),
            (_cells(om, "ros2_1m", 2000, seed_shift=5), 1e-7, 0)]
    print("[gpu] serial reference runs (reactor mode, density held)", flush=True)
    refs = []
    for y0, dt, e in jobs:
        refs.append(_run(gm, om, y0, dt, energy=e))
        torch.cuda.synchronize()
    out = [[None] * 3 for _ in jobs]
    errors = []

    def worker(i):
        try:
            y0, dt, e = jobs[i]
            s = torch.cuda.Stream()
            for r in range(3):
                out[i][r] = _run(gm, om, y0, dt, s, energy=e)
            s.synchronize()
        except Exception as exc:   # reported by the main thread
            errors.append(exc)

    print("[gpu] two threads, two streams, three calls each", flush=True)
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, (ry, rs, rc) in enumerate(refs):
        for y, st, cnt in out[i]:
            assert torch.equal(y, ry) and torch.equal(st, rs) and torch.equal(cnt, rc)
    # the two modes give different states (the reactor mode moved the inert collider)
    inert = np.nonzero(om.inert)[0]
    y_reactor = host_aos(refs[0][0], jobs[0][0].shape[0])
    assert np.abs(y_reactor[:, 1 + inert] / jobs[0][0][:, 1 + inert] - 1.0).max() > 1e-6
    assert np.array_equal(host_aos(refs[1][0], jobs[1][0].shape[0])[:, 1 + inert], jobs[1][0][:, 1 + inert])


def test_rosenbrock_lds_limit_14_species():
    import torch
    from paper_2510_10005_amd import default_options
    from paper_2510_10005_amd._binding import ChemError
    gm, om = gpu_mechanism("mid_14_40")
    with pytest.raises(ChemError, match="LDS"):
        gm.chem_set_launch(1, 0, 256, 0)
    nc = 300
    y0 = _cells(om, "ros2_1m", nc)
    y = dev_soa(y0)
    print("[gpu] autotune, 14 species", flush=True)
    gm.chem_autotune(nc, nc, y, None, default_options(method=1, dt=1e-8, n_steps=0))
    block, grid = gm.chem_get_launch(1, 0)
    assert block in (64, 128) and grid > 0     # 256 lanes would need 186 KB of LDS
    print(f"[gpu] launch {block} x {grid}; integrate", flush=True)
    got, st, cnt = _run(gm, om, y0, 1e-8)
    torch.cuda.synchronize()
    ref = oracle.integrate_ros2(om, y0, 1e-8)
    cnt = cnt.cpu().numpy()
    same = (cnt[0] == ref["accepted"]) & (cnt[1] == ref["rejected"])
    np.testing.assert_array_equal(st.cpu().numpy(), ref["status"])
    assert np.count_nonzero(~same) <= max(1, nc // 50)
    assert integrated_state_error(om, host_aos(got, nc)[same], ref["y"][same]).max() <= 1e-8
