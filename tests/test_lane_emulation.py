"""CPU: the register-resident form's Rosenbrock recording kernel and discrete adjoint kernel, run on
the fiber emulation of a 64-lane wavefront (tests/emu/fiber.hpp, tests/emu/lane_driver.cpp), against
the oracle's adjoint along the same accepted steps.

The whole kernels run as generated (work queue, ballots, the LU with its swap branches,
checkpoint rebuild, segment replay, reverse sweep), with one lane per workgroup (the fiber
emulation needs every lane of a wave at each collective, and on the GPU lanes leave the per-cell
loops at different times) and the cross-lane reduction of the ln A partials replaced by a per-lane
sum.  The case kept here is the P-log mechanism with the adjoint's mechanism functions fully
inlined (CHEM_ADJ_CALL empty), the configuration that computed non-finite gradients on the GPU at
-O3, built with clang -O3, ASan, UBSan and automatic variables filled with a pattern (an
uninitialised read then shows up as a wrong or non-finite value): the kernel matches the oracle
and the sanitizers report nothing.  (Also run while this test was written, with the same result:
-O1 with UBSan, inlined and out of line, and the 10-species mechanism at -O1 and at -O3 with the
sanitizers.)

Bars: the GPU tests' (1e-6 relative: dL/dy0 per component against that component's largest
|value| over the cells and element by element on entries of at least 1e-3 of it; dL/dlnA
against its largest |value| and element by element likewise); step sequences equal.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.sensitivity import ros2_adjoint
from synth import mechanism_file
from synth.states import sample_config

from _gpu import gradient_errors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_10005_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")

BUILDS = {
    "O1-ubsan": ["-O1", "-fsanitize=undefined", "-fno-sanitize-recover=all"],
    "O3-asan-ubsan-pattern": ["-O3", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                              "-ftrivial-auto-var-init=pattern"],
}


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
    d = tmp_path_factory.mktemp("lane_gen")
    gen = str(d / "gen")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, os.path.join(EMU, "gen_main.cpp"),
                    os.path.join(CSRC, "codegen.cpp"), os.path.join(CSRC, "mechanism.cpp"), "-o", gen], check=True)
    return gen


def _driver(generator, d, name, build, inline):
    src = subprocess.run([generator, mechanism_file(name)], capture_output=True, text=True, check=True).stdout
    dyn = "extern __shared__ double chem_dyn_lds[];"
    assert src.count(dyn) == 1
    src = src.replace(dyn, "static double chem_dyn_lds[NU * 256];")   # the dynamic LDS of up to 256 lanes
    red = "__device__ __forceinline__ void block_reduce_grad(GACC& g, double* __restrict__ gpart) {"
    assert src.count(red) == 1
    src = src.replace(red, red + "\n  for (int j = 0; j < NR; ++j) gpart[(i64)blockIdx.x * NR + j] += g[j];\n  return;")
    if inline:
        src = src.replace("#define CHEM_ADJ_CALL __noinline__", "#define CHEM_ADJ_CALL")
    (d / "src.hip").write_text(src)
    exe = str(d / "lane_driver")
    subprocess.run([_clang()] + BUILDS[build] + ["-std=c++20", "-Wno-psabi", "-I", str(d), "-I", EMU,
                                                 os.path.join(EMU, "lane_driver.cpp"), "-o", exe], check=True)
    return exe


# (the other mechanisms' Rosenbrock adjoint runs on the GPU; the sanitized -O3 build of a mechanism
# compiles for about a minute, so the CPU suite keeps the one configuration that needs the host)
CASES = [("plog_12_30", "O3-asan-ubsan-pattern", True)]


@pytest.mark.parametrize("name,build,inline", CASES)
def test_rosenbrock_adjoint_kernel_matches_oracle(generator, tmp_path, name, build, inline):
    om = oracle.load_mechanism(mechanism_file(name))
    if inline and "CHEM_ADJ_CALL __noinline__" not in subprocess.run(
            [generator, mechanism_file(name)], capture_output=True, text=True, check=True).stdout:
        pytest.skip("this mechanism's adjoint is inlined already")
    exe = _driver(generator, tmp_path, name, build, inline)
    nc, ld, dt, K = 4, 7, 4e-9, 8
    T, p, Y = sample_config("ros2_1m", om.ns, nc)
    if name == "plog_12_30":
        p = np.geomspace(2e4, 2e6, nc)          # both intervals of the P-log tables
    y0 = oracle.state_from_TPY(om, T, p, Y)
    lamN = np.random.default_rng(17).standard_normal((nc, om.n)) / np.abs(y0)
    ys, ls = np.zeros((om.n, ld)), np.zeros((om.n, ld))
    ys[:, :nc], ls[:, :nc] = y0.T, lamN.T
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        f.write(ys.astype("<f8").tobytes())
        f.write(np.asarray(om.lnA_default, "<f8").tobytes())
        f.write(ls.astype("<f8").tobytes())
    r = subprocess.run([exe, "ros2adj", str(nc), str(ld), repr(dt), str(K), str(fin), str(fout)],
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    raw = fout.read_bytes()
    n, nr = om.n, om.nr
    o = 0
    y = np.frombuffer(raw[o:o + 8 * n * ld], "<f8").reshape(n, ld)[:, :nc].T
    o += 8 * n * ld
    st = np.frombuffer(raw[o:o + 4 * ld], "<i4")[:nc]
    o += 4 * ld
    acc = np.frombuffer(raw[o:o + 4 * ld], "<i4")[:nc]
    o += 4 * ld
    lam0 = np.frombuffer(raw[o:o + 8 * n * ld], "<f8").reshape(n, ld)[:, :nc].T
    o += 8 * n * ld
    g = np.frombuffer(raw[o:o + 8 * nr], "<f8")
    with np.errstate(all="ignore"):
        ref = oracle.integrate_ros2(om, y0, dt, record=True)
    np.testing.assert_array_equal(st, ref["status"])
    np.testing.assert_array_equal(acc, ref["accepted"])
    assert np.all(np.isfinite(lam0)) and np.all(np.isfinite(g))
    lam0_ref, g_ref = ros2_adjoint(om, lamN, y0, ref["history"])
    col, elem = gradient_errors(lam0, lam0_ref)
    gcol, gelem = gradient_errors(g[None, :], g_ref.sum(axis=0)[None, :])
    print(f"{name} {build} inline={inline}: accepted {acc.tolist()}, dL/dy0 {col:.2e} / {elem:.2e}, "
          f"dL/dlnA {gcol:.2e} / {gelem:.2e}")
    assert max(col, elem, gcol, gelem) <= 1e-6
