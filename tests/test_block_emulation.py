"""CPU: the block form (one cell per 256-thread workgroup, mechanisms with n > 24) against the
oracle and LAPACK, on the fiber emulation of a workgroup (tests/emu/fiber.hpp).

The generated HIP source of a mechanism is compiled for the host with the emulation: the four
wavefronts' lanes are cooperative fibers that switch at every wave collective (shuffle, ballot,
readlane, wave barrier, FP64 matrix-core product, emulated from its documented lane layout) and at
every workgroup barrier; every lane records the source line of the collective it reached, so lanes
of a wave standing at different collectives, or threads at different barriers, stop the run with
exit status 9.  Lanes run one after another between collectives, so a lane that reads LDS another
lane of its wave wrote without a wave barrier in between reads the old value and the results
diverge from the reference.  The build adds UBSan.

Checked: both LU strategies (register panel, LDS panel) with their triangular solves (G x = b,
G^T mu = lam) against LAPACK for the 53-species (factors in LDS) and 150-species (factors in the
device workspace, LDS panel only) sizes,
including a matrix whose first column is tiny (pivoting); backward Euler and the adaptive
Rosenbrock method against the oracle (equal step sequences, states within 1e-8) on the 53-species
mechanism (also the 24-cell, 6 x 1e-8 s configuration, several workgroups on one queue) and on the
30-species SRI/P-log mechanism at both P-log pressure intervals, also with the LDS-panel kernels; the source-term and Jacobian
kernels of the 150-species mechanism against the oracle (1e-12 of the term magnitudes) and its
fixed-step Rosenbrock integration; the backward-Euler discrete adjoint (tape, segment recompute,
halved steps) of all three mechanisms against the oracle's reverse sweep (1e-6).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.integrate import IntegratorOptions
from synth import mechanism_file
from synth.states import paper_sampler, sample_config

from _gpu import integrated_state_error

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_10005_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def generator(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or _clang() is None:
        pytest.skip("no host C++ compilers")
    d = tmp_path_factory.mktemp("block_gen")
    gen = str(d / "gen")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, os.path.join(EMU, "gen_main.cpp"),
                    os.path.join(CSRC, "codegen.cpp"), os.path.join(CSRC, "mechanism.cpp"), "-o", gen], check=True)
    return gen


_built = {}


def _driver(generator, tmp_path_factory, name):
    if name in _built:
        return _built[name]
    d = tmp_path_factory.mktemp(f"block_{name}")
    path = mechanism_file(name)
    with open(d / "src.hip", "w") as f:
        subprocess.run([generator, path], stdout=f, check=True)
    exe = str(d / "driver")
    subprocess.run([_clang(), "-O1", "-std=c++20", "-Wno-psabi", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                    "-I", str(d), "-I", EMU, os.path.join(EMU, "block_driver.cpp"), "-o", exe], check=True)
    _built[name] = (exe, str(d), oracle.load_mechanism(path))
    return _built[name]


def _run(cmd, timeout=900):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, f"emulation failed ({r.returncode}): {r.stderr[-2000:]}"


@pytest.mark.parametrize("name,lus", [("ch4like_53_325", 0), ("ch4like_53_325", 1), ("large_150_1000", 1)])
def test_block_lu_and_solves_match_lapack(generator, tmp_path_factory, name, lus):
    exe, d, om = _driver(generator, tmp_path_factory, name)
    ny = om.n
    rng = np.random.default_rng(7)
    for trial in range(3):
        A = rng.standard_normal((ny, ny))
        if trial == 1:
            A[:, 0] *= 1e-8                      # the first pivot must come from a row swap
        if trial == 2:
            A += 50.0 * np.eye(ny)
        b, lam = rng.standard_normal(ny), rng.standard_normal(ny)
        fin, fout = os.path.join(d, "lu_in.bin"), os.path.join(d, "lu_out.bin")
        with open(fin, "wb") as f:
            f.write(np.concatenate([A.ravel(), b, lam]).astype("<f8").tobytes())
        _run([exe, "lu", fin, fout, str(lus)])
        out = np.frombuffer(open(fout, "rb").read(), "<f8")
        x, mu = out[:ny], out[ny:2 * ny]
        xr, mr = np.linalg.solve(A, b), np.linalg.solve(A.T, lam)
        # backward-stable LU: error within a modest multiple of cond * eps
        bound = 1e3 * np.linalg.cond(A) * np.finfo(float).eps
        assert np.abs(x - xr).max() <= bound * np.abs(xr).max()
        assert np.abs(mu - mr).max() <= bound * np.abs(mr).max()


def _integrate(generator, tmp_path_factory, name, which, cfg, nc, dt, n_steps, ld_pad=3, grid=2, lus=0, energy=0):
    exe, d, om = _driver(generator, tmp_path_factory, name)
    T, p, Y = sample_config(cfg, om.ns, nc)
    if any(rx.kind == "plog" for rx in om.reactions):
        p = np.geomspace(2e4, 2e6, nc)          # both intervals of the P-log tables
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ld = nc + ld_pad
    ys = np.zeros((om.n, ld))
    ys[:, :nc] = y0.T
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fin, "wb") as f:
        f.write(ys.astype("<f8").tobytes())
        f.write(np.asarray(om.lnA_default, "<f8").tobytes())
    _run([exe, which, str(nc), str(ld), repr(dt), str(n_steps), fin, fout, str(grid), str(lus), str(energy)])
    raw = open(fout, "rb").read()
    k = 8 * om.n * ld
    y = np.frombuffer(raw[:k], "<f8").reshape(om.n, ld)[:, :nc].T
    st = np.frombuffer(raw[k:k + 4 * ld], "<i4")[:nc]
    cnt = np.frombuffer(raw[k + 4 * ld:], "<i4").reshape(3, ld)[:, :nc]
    return om, y0, y, st, cnt


@pytest.mark.parametrize("name,lus", [("ch4like_53_325", 0), ("mix_30_90", 0), ("ch4like_53_325", 1)])
def test_block_backward_euler_matches_oracle(generator, tmp_path_factory, name, lus):
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, name, "be", "be_small", 3, 2e-8, 2, lus=lus)
    ref = oracle.integrate_be(om, y0, 2e-8, 2)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["steps"])
    assert int(cnt[2].sum()) == int(ref["newton"].sum())
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8


def test_block_backward_euler_recorded_geometry(generator, tmp_path_factory):
    """24 cells, 6 steps of 1e-8 s, ld = 29, four workgroups on one queue (the configuration whose
    run with the earlier one-wavefront-per-cell kernels did not complete on the GPU)."""
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, "ch4like_53_325", "be", "be_small", 24, 6e-8, 6,
                                    ld_pad=5, grid=4)
    ref = oracle.integrate_be(om, y0, 6e-8, 6)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["steps"])
    assert int(cnt[2].sum()) == int(ref["newton"].sum())
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8


@pytest.mark.parametrize("name,lus", [("ch4like_53_325", 0), ("mix_30_90", 1)])
def test_block_rosenbrock_matches_oracle(generator, tmp_path_factory, name, lus):
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, name, "ros2", "ros2_methane", 3, 1e-9, 0, lus=lus)
    ref = oracle.integrate_ros2(om, y0, 1e-9)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["accepted"])
    np.testing.assert_array_equal(cnt[1], ref["rejected"])
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8


@pytest.mark.parametrize("name,lus", [("ch4like_53_325", 0), ("mix_30_90", 1)])
def test_block_reactor_backward_euler_matches_oracle(generator, tmp_path_factory, name, lus):
    """Constant-pressure reactor form (energy 2): the dilatation terms of the sources and of every
    Jacobian the Newton iterations factor."""
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, name, "be", "be_small", 3, 2e-8, 2, lus=lus,
                                    energy=oracle.CONST_P_REACTOR)
    ref = oracle.integrate_be(om, y0, 2e-8, 2, opt=IntegratorOptions(energy=oracle.CONST_P_REACTOR))
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["steps"])
    assert int(cnt[2].sum()) == int(ref["newton"].sum())
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8
    # the reactor form changes the density, and the held-density run differs from it
    held = oracle.integrate_be(om, y0, 2e-8, 2)
    assert integrated_state_error(om, y, held["y"]).max() > 1e-6


@pytest.mark.parametrize("name,lus", [("ch4like_53_325", 1)])
def test_block_reactor_rosenbrock_matches_oracle(generator, tmp_path_factory, name, lus):
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, name, "ros2", "ros2_methane", 3, 1e-9, 0, lus=lus,
                                    energy=oracle.CONST_P_REACTOR)
    ref = oracle.integrate_ros2(om, y0, 1e-9, opt=IntegratorOptions(energy=oracle.CONST_P_REACTOR))
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["accepted"])
    np.testing.assert_array_equal(cnt[1], ref["rejected"])
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8


@pytest.mark.parametrize("energy", [0, 2])
def test_block_api_kernels_150_species(generator, tmp_path_factory, energy):
    exe, d, om = _driver(generator, tmp_path_factory, "large_150_1000")
    nc, ld = 3, 5
    T, p, Y = paper_sampler(om.ns, nc, 21)
    y = oracle.state_from_TPY(om, T, p, Y)
    ys = np.zeros((om.n, ld))
    ys[:, :nc] = y.T
    fin, fout = os.path.join(d, "api_in.bin"), os.path.join(d, "api_out.bin")
    with open(fin, "wb") as f:
        f.write(ys.astype("<f8").tobytes())
        f.write(np.asarray(om.lnA_default, "<f8").tobytes())
    _run([exe, "jac", str(nc), str(ld), fin, fout, str(energy)])
    raw = np.frombuffer(open(fout, "rb").read(), "<f8")
    S = raw[:om.n * ld].reshape(om.n, ld)[:, :nc].T
    J = raw[om.n * ld:].reshape(nc, om.n, om.n)
    Sref = oracle.source_terms(om, y, None, energy)
    den = np.abs(Sref) + oracle.source_sum_scale(om, y, None, energy)
    assert (np.abs(S - Sref) / np.where(den > 0, den, 1.0)).max() <= 1e-12
    Jref, M = oracle.jacobian(om, y, None, energy, magnitude=True)
    den = np.abs(Jref) + M
    assert (np.abs(J - Jref) / np.where(den > 0, den, 1.0)).max() <= 1e-12


def test_block_rosenbrock_150_species(generator, tmp_path_factory):
    """Fixed-step Rosenbrock (4 steps of 1e-12 s): every attempt is accepted, so the oracle needs
    only four Jacobians of the 151 x 151 system per cell."""
    om, y0, y, st, cnt = _integrate(generator, tmp_path_factory, "large_150_1000", "ros2", "ros2_large", 2, 4e-12, 4)
    ref = oracle.integrate_ros2(om, y0, 4e-12, fixed_steps=4)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(cnt[0], ref["accepted"])
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8


@pytest.mark.parametrize("name,step,nc,cfg,energy", [("ch4like_53_325", 1e-6, 3, "be_small", 0),
                                                     ("mix_30_90", 1e-3, 3, "be_small", 0),
                                                     ("large_150_1000", 1e-11, 1, "ros2_large", 0),
                                                     ("mix_30_90", 1e-5, 3, "be_small", 2)])
def test_block_be_adjoint_matches_oracle(generator, tmp_path_factory, name, step, nc, cfg, energy):
    """Backward Euler with a tape (checkpoints every 2 steps, 3 steps: for the two smaller mechanisms
    a halved step and a partial last segment), then the block-form discrete adjoint against the
    oracle's reverse sweep along the oracle's recorded (sub)steps; the 150-species mechanism keeps
    its factors in the device workspace."""
    from oracle.sensitivity import be_adjoint, final_loss
    from synth.states import loss_weights
    exe, d, om = _driver(generator, tmp_path_factory, name)
    ld, grid = nc + 2, 2
    dt, n_steps, K = 3 * step, 3, 2
    T, p, Y = sample_config(cfg, om.ns, nc)
    if any(rx.kind == "plog" for rx in om.reactions):
        p = np.geomspace(2e4, 2e6, nc)
    y0 = oracle.state_from_TPY(om, T, p, Y)
    ref = oracle.integrate_be(om, y0, dt, n_steps, record=True, opt=IntegratorOptions(energy=energy))
    if om.ns < 100:
        assert max(len(t) for t in ref["trajectory"]) > n_steps  # at least one halved step
    _, lamN = final_loss(om, ref["y"], loss_weights(nc, om.ns))
    ys, ls = np.zeros((om.n, ld)), np.zeros((om.n, ld))
    ys[:, :nc], ls[:, :nc] = y0.T, lamN.T
    fin, fout = os.path.join(d, "adj_in.bin"), os.path.join(d, "adj_out.bin")
    with open(fin, "wb") as f:
        f.write(ys.astype("<f8").tobytes())
        f.write(np.asarray(om.lnA_default, "<f8").tobytes())
        f.write(ls.astype("<f8").tobytes())
    _run([exe, "adj", str(nc), str(ld), repr(dt), str(n_steps), str(K), fin, fout, str(grid), str(energy)])
    raw = open(fout, "rb").read()
    k = 8 * om.n * ld
    y = np.frombuffer(raw[:k], "<f8").reshape(om.n, ld)[:, :nc].T
    st = np.frombuffer(raw[k:k + 4 * ld], "<i4")[:nc]
    lam0 = np.frombuffer(raw[k + 4 * ld:2 * k + 4 * ld], "<f8").reshape(om.n, ld)[:, :nc].T
    g = np.frombuffer(raw[2 * k + 4 * ld:], "<f8")
    np.testing.assert_array_equal(st, ref["status"])
    assert integrated_state_error(om, y, ref["y"]).max() <= 1e-8
    lam0_ref, g_ref = be_adjoint(om, lamN, ref["trajectory"], energy=energy)
    scale = np.abs(lam0_ref).max(axis=0, keepdims=True)
    assert (np.abs(lam0 - lam0_ref) / np.where(scale > 0, scale, 1.0)).max() <= 1e-6
    gs = g_ref.sum(axis=0)
    assert (np.abs(g - gs) / np.abs(gs).max()).max() <= 1e-6
