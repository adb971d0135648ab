"""GPU: the CFD coupling entry points against the oracle (oracle.coupling).

* chem_T_from_energy: temperatures after 1, 2 and 5 Newton iterations from guesses up to 300 K
  away, both energy modes (rho u, rho h), on every test mechanism including the 53-species one,
  within 1e-12 relative of the oracle's iterates (the same fixed-count iteration; the energies
  are sums of a few terms of like sign, so they are well conditioned); a ragged cell count with
  ld > n; sampled cells of the 1,048,576-cell state set; empty batch; argument errors.
* chem_cfd_source: R_i = W_i (C^{n+1} - C^n)/dt elementwise within 1e-13 of max |R_i| per species.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle.coupling import T_from_energy, energy_density, openfoam_source
from synth.states import STATE_CONFIGS, sample_config, sample_states

from _gpu import dev_soa, gpu_mechanism, host_aos

pytestmark = pytest.mark.gpu

MECHS = ["tiny_5_6", "tiny_8_14", "h2like_10_27", "ch4like_53_325"]


@pytest.fixture(scope="module", params=MECHS)
def mechs(request):
    print(f"[gpu] loading {request.param}", flush=True)
    return gpu_mechanism(request.param)


@pytest.mark.parametrize("energy", [0, 1])
@pytest.mark.parametrize("n_iter", [1, 2, 5])
def test_T_from_energy_matches_oracle(mechs, energy, n_iter):
    gm, om = mechs
    nc = 333
    ld = nc + 11
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    y = oracle.state_from_TPY(om, T, p, Y)
    C, Tstar = y[:, 1:], y[:, 0]
    e, _ = energy_density(om, C, Tstar, energy)
    T0 = Tstar + np.random.default_rng(9).uniform(-300.0, 300.0, nc)
    ref = T_from_energy(om, C, e, T0, energy, n_iter)
    print(f"[gpu] {om.ns} species: T from energy, mode {energy}, {n_iter} iterations", flush=True)
    Tout = torch.full((ld,), float("nan"), dtype=torch.float64, device="cuda")
    gm.chem_T_from_energy(nc, ld, dev_soa(C, ld), dev_soa(e, ld)[0], dev_soa(T0, ld)[0], energy, n_iter, Tout)
    torch.cuda.synchronize()
    got = Tout.cpu().numpy()
    np.testing.assert_allclose(got[:nc], ref, rtol=1e-12)
    assert np.all(np.isnan(got[nc:]))
    if n_iter == 5:
        np.testing.assert_allclose(got[:nc], Tstar, rtol=1e-12)


def test_T_from_energy_in_place_and_edges(mechs):
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    nc = 64
    T, p, Y = sample_config("be_small", om.ns, nc)
    y = oracle.state_from_TPY(om, T, p, Y)
    e, _ = energy_density(om, y[:, 1:], y[:, 0], 1)
    yd = dev_soa(y, nc)
    Td = dev_soa(y[:, 0] + 150.0, nc)[0]
    ed = dev_soa(e, nc)[0]
    gm.chem_T_from_energy(nc, nc, yd[1:], ed, Td, 1, 5, Td)      # C = species rows of y; T in place
    torch.cuda.synchronize()
    np.testing.assert_allclose(Td.cpu().numpy(), y[:, 0], rtol=1e-12)
    gm.chem_T_from_energy(0, 0, yd[1:], ed, Td, 1, 5, Td)
    with pytest.raises(ChemError, match="n_iter"):
        gm.chem_T_from_energy(nc, nc, yd[1:], ed, Td, 1, 0, Td)
    with pytest.raises(ChemError, match="energy"):
        gm.chem_T_from_energy(nc, nc, yd[1:], ed, Td, 7, 5, Td)
    with pytest.raises(ChemError, match="null"):
        gm.chem_T_from_energy(nc, nc, None, ed, Td, 1, 5, Td)


def test_cfd_source_matches_oracle(mechs):
    from paper_2510_10005_amd._binding import ChemError
    gm, om = mechs
    nc = 257
    ld = nc + 3
    T, p, Y = sample_config("be_small", om.ns, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    rng = np.random.default_rng(4)
    y1 = y0 * (1.0 + 1e-3 * rng.standard_normal(y0.shape))
    dt = 1e-7
    ref = openfoam_source(om, y0, y1, dt)
    R = torch.full((om.ns, ld), float("nan"), dtype=torch.float64, device="cuda")
    gm.chem_cfd_source(nc, ld, dev_soa(y0, ld), dev_soa(y1, ld), dt, R)
    torch.cuda.synchronize()
    got = host_aos(R, nc)
    scale = np.abs(ref).max(axis=0, keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    assert torch.isnan(R[:, nc:]).all()
    with pytest.raises(ChemError, match="dt"):
        gm.chem_cfd_source(nc, ld, dev_soa(y0, ld), dev_soa(y1, ld), 0.0, R)


def test_T_from_energy_fullsize_sampled():
    """The 1,048,576-cell state set (h2like): rho u from the true T, guesses 200 K low, 5 iterations;
    64 seeded cells against the oracle."""
    gm, om = gpu_mechanism("h2like_10_27")
    cfg = STATE_CONFIGS["ros2_1m"]
    n = cfg.n_cells
    T, p, Y = sample_states(om.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    y = oracle.state_from_TPY(om, T, p, Y)
    idx = np.random.default_rng(6).choice(n, size=64, replace=False)
    e = energy_density(om, y[:, 1:], y[:, 0], 1)[0]
    T0 = y[:, 0] - 200.0
    print("[gpu] T from energy over 1,048,576 cells", flush=True)
    yd = dev_soa(y, n)
    Tout = torch.empty(n, dtype=torch.float64, device="cuda")
    gm.chem_T_from_energy(n, n, yd[1:], dev_soa(e, n)[0], dev_soa(T0, n)[0], 1, 5, Tout)
    torch.cuda.synchronize()
    ref = T_from_energy(om, y[idx, 1:], e[idx], T0[idx], 1, 5)
    np.testing.assert_allclose(Tout.cpu().numpy()[idx], ref, rtol=1e-12)
