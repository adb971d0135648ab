"""CPU: the generated vector-Jacobian product of the Rosenbrock adjoint against the oracle.

The generated mechanism functions of the register-resident form (prelude + mechanism block) are
compiled for the host (tests/emu/vjp_driver.cpp) and mech_vjp is evaluated on seeded states:

* with plain numbers: J(y)^T u and u^T dS/dlnA(y) against the oracle's analytic Jacobian and
  dS/dlnA;
* with dual numbers y + eps d: the value parts again, and the dual parts against complex-step
  directional derivatives of the oracle's Jacobian and dS/dlnA along d ((J'(y)[d])^T u and
  u^T (dS/dlnA)'(y)[d]), which the adjoint's second-derivative terms use.
Each case is built twice: g++ -O1, and clang -O3 with ASan, UBSan and automatic variables filled
with a pattern (so an uninitialised read would show as a wrong or non-finite value).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.kinetics import dsource_dlnA, jacobian
from synth import mechanism_file
from synth.states import sample_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_10005_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
MARK = "// ------------------------------------------------------------------ matrix storage"


@pytest.fixture(scope="module")
def generator(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("vjp_gen")
    gen = str(d / "gen")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, os.path.join(EMU, "gen_main.cpp"),
                    os.path.join(CSRC, "codegen.cpp"), os.path.join(CSRC, "mechanism.cpp"), "-o", gen], check=True)
    return cxx, gen


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


# build variants: g++ -O1; clang -O3 with AddressSanitizer, UndefinedBehaviorSanitizer and every
# automatic variable pre-filled with a pattern (an uninitialised read then shows up as a wrong or
# non-finite value instead of a benign leftover)
BUILDS = {
    "gcc-O1": None,
    "clang-O3-asan-ubsan-pattern": ["-O3", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                    "-ftrivial-auto-var-init=pattern"],
}


def _build(generator, tmp_path, name, build="gcc-O1"):
    cxx, gen = generator
    path = mechanism_file(name)
    src = subprocess.run([gen, path], capture_output=True, text=True, check=True).stdout
    (tmp_path / "mech_block.hip").write_text(src[:src.index(MARK)])
    exe = str(tmp_path / "vjpd")
    flags = BUILDS[build]
    if flags is None:
        cmd = [cxx, "-O1"]
    else:
        cl = _clang()
        if cl is None:
            pytest.skip("no clang++")
        cmd = [cl] + flags
    subprocess.run(cmd + ["-std=c++17", "-Wno-unknown-pragmas", "-include", "cstdlib", "-I", str(tmp_path),
                          os.path.join(EMU, "vjp_driver.cpp"), "-o", exe], check=True)
    return exe, oracle.load_mechanism(path)


@pytest.mark.parametrize("build", list(BUILDS))
@pytest.mark.parametrize("name", ["tiny_8_14", "h2like_10_27", "sri_12_30", "plog_12_30"])
@pytest.mark.parametrize("energy", [0, 1])
def test_vjp_matches_oracle(generator, tmp_path, name, energy, build):
    exe, m = _build(generator, tmp_path, name, build)
    nc = 6
    T, p, Y = sample_config("ros2_1m", m.ns, nc)
    y = oracle.state_from_TPY(m, T, p, Y)
    rng = np.random.default_rng(42)
    u = rng.standard_normal((nc, m.n)) / np.abs(y)
    d = rng.standard_normal((nc, m.n)) * np.abs(y) * 1e-2
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        f.write(np.int32(nc).tobytes())
        f.write(np.asarray(m.lnA_default, "<f8").tobytes())
        for c in range(nc):
            f.write(np.concatenate([y[c], u[c], d[c]]).astype("<f8").tobytes())
    subprocess.run([exe, str(energy), str(fin), str(fout)], check=True, timeout=120)
    raw = np.frombuffer(fout.read_bytes(), "<f8").reshape(nc, -1)
    n, nr = m.n, m.nr
    v, g = raw[:, :n], raw[:, n:n + nr]
    vv, vd = raw[:, n + nr:2 * n + nr], raw[:, 2 * n + nr:3 * n + nr]
    g1, g2 = raw[:, 3 * n + nr:3 * n + 2 * nr], raw[:, 3 * n + 2 * nr:]

    J, Mg = jacobian(m, y, energy=energy, magnitude=True)
    P = dsource_dlnA(m, y, energy=energy)
    h = 1e-40
    dJ = np.imag(jacobian(m, y + 1j * h * d, energy=energy)) / h
    dP = np.imag(dsource_dlnA(m, y + 1j * h * d, energy=energy)) / h
    v_ref = np.einsum("cik,ci->ck", J, u)
    scale = np.einsum("cik,ci->ck", Mg, np.abs(u))     # bound on the rounding of each component
    assert np.all(np.abs(v - v_ref) <= 1e-12 * scale + 1e-300)
    assert np.all(np.abs(vv - v_ref) <= 1e-12 * scale + 1e-300)
    g_ref = np.einsum("cij,ci->cj", P, u)
    g_scale = np.einsum("cij,ci->cj", np.abs(P), np.abs(u))
    assert np.all(np.abs(g - g_ref) <= 1e-12 * g_scale + 1e-300)
    vd_ref = np.einsum("cik,ci->ck", dJ, u)
    gd_ref = np.einsum("cij,ci->cj", dP, u)
    for c in range(nc):
        assert np.max(np.abs(vd[c] - vd_ref[c])) <= 1e-10 * np.max(np.abs(vd_ref[c])), c
        assert np.max(np.abs(g2[c] - gd_ref[c])) <= 1e-10 * np.max(np.abs(gd_ref[c])), c
        assert np.max(np.abs(g1[c] - (g_ref[c] + gd_ref[c]))) <= 1e-10 * np.max(np.abs(g_ref[c] + gd_ref[c])), c
