#!/usr/bin/env python3
"""Benchmark: batched FP64 chemistry integration on one MI355X.

Workload (one "step" = one operator-split step over the whole batch): the 10-species /
27-reaction synthetic mechanism, 1,048,576 constant-pressure cells with T0 ~ U[900, 2400] K and
Dirichlet(0.5) mass fractions at 101325 Pa, integrated over dt = 1e-6 s with the adaptive
two-stage Rosenbrock method (rtol 1e-6, atol 1e-10) in the persistent work-queue form.  Each
step restarts from the same initial states, which are resident in device memory.

Printed (one JSON line): cell-substeps/s (accepted Rosenbrock steps of all cells per second),
the roofline position of the integration kernel (algorithmic FP64 flops per launch over its
event-timed duration against the FP64 vector peak), the plain one-launch-per-substep form on
the same cells, the backward-Euler adjoint/forward time ratio, and the CPU oracle's rate on a
bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNEL_CACHE = os.path.join(ROOT, "_build", "kernels")
PEAK_FP64 = 78.6e12          # MI355X FP64 vector peak, FLOP/s (256 CU x 128 flop/clk x 2.4 GHz)
PEAK_HBM = 8.0e12            # bytes/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", default="", help="block,grid of the persistent kernel (skips autotuning)")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--skip-adjoint", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-kernels", action="store_true")
    ap.add_argument("--skip-large", action="store_true", help="skip the 53- and 150-species mechanism legs")
    ap.add_argument("--skip-reactor", action="store_true", help="skip the constant-pressure reactor-mode leg")
    ap.add_argument("--c2-cells", type=int, default=4096,
                    help="cells of the 53-species Rosenbrock state set integrated over 1e-5 s (262144 = all)")
    ap.add_argument("--probe", type=int, default=None,
                    help="probe_attempts of the persistent form (default: the library's)")
    ap.add_argument("--cpu-cells", type=int, default=128, help="oracle cells per host process")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the batched chemistry path here is single-device "
              "(cells shard trivially across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_10005_amd import (CHEM_BE, CHEM_PERSISTENT, CHEM_PLAIN, CHEM_ROS2, CHEM_SDIRK2, CHEM_SDIRK4,
                                      Mechanism, Tape,
                                      default_options)
    from paper_2510_10005_amd.flops import MechanismCounts
    from synth import mechanism_file
    from synth.states import STATE_CONFIGS, loss_weights, sample_states

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    path = mechanism_file("h2like_10_27")
    gm = Mechanism(path, KERNEL_CACHE)
    counts = MechanismCounts(path)
    cfg = STATE_CONFIGS["ros2_1m"]
    n = args.cells
    log(f"drawing {n} states")
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    counters = torch.zeros((3, n), dtype=torch.int32, device=dev)
    probe = {} if args.probe is None else {"probe_attempts": args.probe}
    opts = default_options(method=CHEM_ROS2, dt=1e-6, n_steps=0, rtol=1e-6, atol=1e-10, form=CHEM_PERSISTENT, **probe)

    if args.launch:
        b_, g_ = (int(v) for v in args.launch.split(","))
        gm.chem_set_launch(CHEM_ROS2, CHEM_PERSISTENT, b_, g_)
    elif not args.no_autotune:
        nt = min(n, 1 << 17)
        log(f"autotuning the persistent launch on {nt} cells")
        gm.chem_autotune(nt, n, y0, None, opts)
    block, grid = gm.chem_get_launch(CHEM_ROS2, CHEM_PERSISTENT)
    log(f"persistent launch: block {block}, grid {grid}")

    def one_step(form):
        y.copy_(y0)
        o = default_options(method=CHEM_ROS2, dt=1e-6, n_steps=0, rtol=1e-6, atol=1e-10, form=form, **probe)
        gm.chem_integrate(n, n, y, None, o, None, status, counters)

    for _ in range(args.warmup):
        one_step(CHEM_PERSISTENT)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    acc_total = 0
    att_total = 0
    kernel_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        y.copy_(y0)
        ev[k][0].record(stream)
        gm.chem_integrate(n, n, y, None, opts, None, status, counters)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # every timed step integrates the same cells, so the last step's counters hold each step's work
    acc = int(counters[0].sum().item())
    rej = int(counters[1].sum().item())
    acc_total = acc * args.steps
    att_total = (acc + rej) * args.steps
    kernel_ms = sum(a.elapsed_time(b) for a, b in ev)
    n_fail = int((status != 0).sum().item())
    value = acc_total / wall
    per_attempt = counts.ros2_attempt()
    achieved = per_attempt.flops * att_total / (kernel_ms * 1e-3)
    log(f"persistent: {acc} accepted + {rej} rejected substeps per step, {wall / args.steps * 1e3:.1f} ms/step, "
        f"{value:.3e} cell-substeps/s, {achieved / 1e12:.2f} TFLOP/s algorithmic, failed cells {n_fail}")
    sub = counters[0].to(torch.float64)
    imbalance = float(sub.max().item() / max(1.0, sub.median().item()))
    # the persistent result of the timed steps, for the oracle's parity check on its subset
    gpu_result = None if args.skip_cpu else (y.cpu().numpy(), counters.cpu().numpy())

    extras = {"persistent_launch": {"block": block, "grid": grid, "probe_attempts": opts.probe_attempts},
              "accepted_substeps_per_step": acc, "rejected_attempts_per_step": rej,
              "substep_max_over_median": imbalance, "failed_cells": n_fail,
              "flops_per_attempt": per_attempt.flops, "transcendentals_per_attempt": per_attempt.tops,
              "transcendentals_per_s": per_attempt.tops * att_total / (kernel_ms * 1e-3)}

    extras["graph_replay"] = graph_replay_rate(gm, torch, n, y, y0, opts, status, counters, acc)

    if not args.skip_kernels:
        extras["api_kernels"] = api_kernel_rates(gm, counts, y0, n, torch, dev)

    if not args.skip_plain:
        torch.cuda.synchronize()
        tp = time.perf_counter()
        one_step(CHEM_PLAIN)
        torch.cuda.synchronize()
        wp = time.perf_counter() - tp
        acc_p = int(counters[0].sum().item())
        extras["plain_form"] = {"cell_substeps_per_s": acc_p / wp, "ms_per_step": wp * 1e3,
                                "persistent_speedup": value / (acc_p / wp)}
        log(f"plain: {acc_p / wp:.3e} cell-substeps/s ({wp * 1e3:.1f} ms); persistent speedup {value / (acc_p / wp):.2f}x")

    if not args.skip_reactor:
        extras["reactor_mode"] = reactor_mode_rate(gm, torch, n, y, y0, status, counters, probe, value)

    extras["be_1024"] = be_small_rate(gm, torch, np, dev, default_options, CHEM_BE, sample_states, STATE_CONFIGS)
    for name, method in (("sdirk2_1024", CHEM_SDIRK2), ("sdirk4_1024", CHEM_SDIRK4)):
        extras[name] = sdirk_small_rate(gm, counts, method, torch, np, dev, default_options, sample_states,
                                        STATE_CONFIGS)
    for name, solver in (("yass_lu_1024", 0), ("yass_gmres_1024", 1)):
        extras[name] = yass_small_rate(gm, counts, solver, torch, np, dev, default_options, sample_states,
                                       STATE_CONFIGS)

    if not args.skip_adjoint:
        # the differentiation workload: 53-species mechanism, 16,384 cells, 500 x 2e-8 s, checkpoints every 50
        gm53 = Mechanism(mechanism_file("ch4like_53_325"), KERNEL_CACHE)
        c3 = STATE_CONFIGS["adjoint_methane"]
        extras["adjoint"] = adjoint_ratio(gm53, torch, np, dev, Tape, default_options, CHEM_BE, sample_states,
                                          loss_weights, STATE_CONFIGS, mech_name="ch4like_53_325",
                                          T_range=c3.T_range, alpha=c3.alpha, reps=1)
        del gm53
        extras["adjoint_h2like_10_27"] = adjoint_ratio(gm, torch, np, dev, Tape, default_options, CHEM_BE,
                                                       sample_states, loss_weights, STATE_CONFIGS)

        extras["adjoint_rosenbrock"] = ros2_adjoint_ratio(gm, torch, np, dev, Tape, default_options, sample_states,
                                                          loss_weights, cfg)

    if not args.skip_large:
        legs = large_mechanism_legs(torch, np, dev, args)
        extras["large_150_1000"] = legs.pop("large_150_1000")
        extras["ch4like_53_325"] = legs

    cpu = None
    if not args.skip_cpu:
        # the timed steps all integrate the same cells: y and counters hold the last step's result
        cpu = cpu_baseline(path, args.cpu_cells, cfg, T, p, Y, *gpu_result)

    line = {
        "metric": "FP64 cell-substeps/sec + fraction of FP64 roofline; adjoint/forward time ratio",
        "value": value,
        "unit": "cell-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ros2_1m: 10-species/27-reaction synthetic mechanism, {n} constant-pressure cells, "
                               "T0~U[900,2400] K, Dirichlet(0.5) mass fractions, adaptive 2-stage Rosenbrock "
                               "(rtol 1e-6, atol 1e-10) over one 1e-6 s split step, persistent work-queue kernel; "
                               "rate draws ln A ~ U[20,35] read in (cm, mol, s) units with T^b referenced to 1000 K",
                   "cells": n, "mechanism": "h2like_10_27", "method": "ros2", "dt_s": 1e-6,
                   "lnA_reading": "U[20,35] in cm-mol-s units at a 1000 K reference for T^b (stored in SI-kmol)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64, "traffic": measured_traffic(path),
                     "kernel": "chem_k_ros2_persistent", "kernel_ms_per_launch": kernel_ms / args.steps},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


def reactor_mode_rate(gm, torch, n, y, y0, status, counters, probe, value_held):
    """The headline workload in the constant-pressure reactor mode (energy 2), whose density change
    moves every species: the register form's full-system build solves for T and all ten species
    (eleven components instead of ten).  One warm-up call (it also loads that build), then one
    timed split step.  Its parity with the oracle is covered by the GPU tests."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, default_options
    o = default_options(method=CHEM_ROS2, dt=1e-6, n_steps=0, rtol=1e-6, atol=1e-10, form=CHEM_PERSISTENT,
                        energy=2, **probe)
    y.copy_(y0)
    gm.chem_integrate(n, n, y, None, o, None, status, counters)
    y.copy_(y0)
    torch.cuda.synchronize()
    a = time.perf_counter()
    gm.chem_integrate(n, n, y, None, o, None, status, counters)
    torch.cuda.synchronize()
    w = time.perf_counter() - a
    acc = int(counters[0].sum().item())
    rej = int(counters[1].sum().item())
    fails = int((status != 0).sum().item())
    log(f"reactor mode: {acc} accepted + {rej} rejected substeps in {w * 1e3:.1f} ms, {acc / w:.3e} cell-substeps/s "
        f"({acc / w / value_held:.2f} of the density-holding mode's rate), failed cells {fails}")
    return {"workload": "the headline cells and step in energy mode 2 (constant-pressure reactor), full-system build",
            "ms": w * 1e3, "accepted_substeps": acc, "rejected_attempts": rej, "cell_substeps_per_s": acc / w,
            "rate_over_density_holding": acc / w / value_held, "failed_cells": fails}


def graph_replay_rate(gm, torch, n, y, y0, opts, status, counters, acc_eager):
    """The split step (state reset + chem_integrate: probe launch, bin scan, scatter, resume launch)
    captured once in a HIP graph and replayed: 2 untimed replays, then the median of 10 replays
    timed with events on the replay stream; the replayed states must equal the eager step's."""
    y_ref = y.clone()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        y.copy_(y0)
        gm.chem_integrate(n, n, y, None, opts, None, status, counters)
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(y, y_ref))
    ms = []
    stream = torch.cuda.current_stream()
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    med = 0.5 * (ms[4] + ms[5])
    acc = int(counters[0].sum().item())
    log(f"graph replay: median {med:.1f} ms of 10 (min {ms[0]:.1f}, max {ms[-1]:.1f}), {acc / (med * 1e-3):.3e} "
        f"cell-substeps/s, states equal to the eager step: {same}")
    del g
    return {"ms_median_of_10": med, "ms_min": ms[0], "ms_max": ms[-1], "cell_substeps_per_s": acc / (med * 1e-3),
            "accepted_substeps": acc, "states_equal_eager": same, "accepted_equal_eager": acc == acc_eager}


def kernel_code_sha256(hsaco_path, symbol):
    """SHA-256 of one kernel's machine code in a code object (ELF64: the function symbol's bytes
    in its section), so that a profile stays attached to exactly the code it measured."""
    import hashlib
    import struct
    with open(hsaco_path, "rb") as f:
        b = f.read()
    shoff, = struct.unpack_from("<Q", b, 0x28)
    shentsize, shnum = struct.unpack_from("<HH", b, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", b, shoff + i * shentsize) for i in range(shnum)]
    for sec in secs:
        if sec[1] != 2:           # SHT_SYMTAB
            continue
        strtab = secs[sec[6]]
        for k in range(sec[5] // 24):
            name_off, info, other, shndx, value, size = struct.unpack_from("<IBBHQQ", b, sec[4] + k * 24)
            start = strtab[4] + name_off
            name = b[start:b.index(b"\0", start)].decode()
            if name == symbol and (info & 0xF) == 2:       # STT_FUNC
                text = secs[shndx]
                off = text[4] + (value - text[3])
                return hashlib.sha256(b[off:off + size]).hexdigest()
    raise KeyError(symbol)


def measured_traffic(mech_path):
    """HBM bytes per split step of the integration kernel from the committed rocprofv3 record
    (FETCH_SIZE and WRITE_SIZE, calibrated against a copy kernel), or None when the kernel's
    machine code differs from the code that was profiled."""
    from paper_2510_10005_amd._binding import precompile
    rec_path = os.path.join(ROOT, "profiles", "ros2_persistent_h2like_1m_traffic.json")
    if not os.path.exists(rec_path):
        return None
    with open(rec_path) as f:
        rec = json.load(f)
    if "kernel" not in rec or "kernel_code_sha256" not in rec:
        log("traffic: the profile record names no kernel code hash; reporting null")
        return None
    code = precompile(mech_path, KERNEL_CACHE)
    digest = kernel_code_sha256(code, rec["kernel"])
    if digest != rec["kernel_code_sha256"]:
        log(f"traffic: {rec['kernel']} in {os.path.basename(code)} is not the profiled code "
            f"({digest[:12]} vs {rec['kernel_code_sha256'][:12]}); reporting null")
        return None
    return rec["bytes_per_step"]


def api_kernel_rates(gm, counts, y0, n, torch, dev, reps=5):
    """Standalone source-term and Jacobian kernels over the same cells: event-timed per launch,
    algorithmic FP64 rate against the vector peak and HBM bytes (state in, result out) against
    the HBM peak."""
    nn = gm.n
    stream = torch.cuda.current_stream()
    out = {}
    src = torch.empty((nn, n), dtype=torch.float64, device=dev)
    jac = torch.empty((nn * nn, n), dtype=torch.float64, device=dev)
    cases = (("source_terms", lambda: gm.chem_source_terms(n, n, y0, None, 0, src), counts.source(), 2 * nn * 8),
             ("jacobian", lambda: gm.chem_jacobian(n, n, y0, None, 0, jac), counts.jacobian(), (nn + nn * nn) * 8))
    for name, fn, c, nbytes in cases:
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) * 1e-3 / reps
        fl = c.flops * n / sec
        bw = nbytes * n / sec
        out[name] = {"ms_per_launch": sec * 1e3, "cells": n, "flops_per_cell": c.flops,
                     "transcendentals_per_cell": c.tops, "tflops_algorithmic": fl / 1e12,
                     "fp64_frac": fl / PEAK_FP64, "hbm_bytes_per_cell": nbytes, "hbm_gbs": bw / 1e9,
                     "hbm_frac": bw / PEAK_HBM, "transcendentals_per_s": c.tops * n / sec}
        log(f"{name}: {sec * 1e3:.3f} ms per launch, {fl / 1e12:.2f} TFLOP/s algorithmic ({fl / PEAK_FP64:.1%}), "
            f"{bw / 1e9:.0f} GB/s ({bw / PEAK_HBM:.1%} of HBM)")
    del src, jac
    return out


def sdirk_small_rate(gm, counts, method, torch, np, dev, default_options, sample_states, STATE_CONFIGS):
    """SDIRK-2 (Appendix A.1) or SDIRK-4 (Appendix A.2) on the 1,024-cell workload's states over its
    2e-5 s in 100 steps of 2e-7 s, persistent form, autotuned launch.  (At the paper's steps, 7e-7 s
    and 1e-6 s, Table 5, Newton fails in about 15 % and 20 % of the cells of this synthetic
    mechanism; the SDIRK schemes have no halving.)"""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_SDIRK2
    label, stages = ("SDIRK-2", 2) if method == CHEM_SDIRK2 else ("SDIRK-4", 5)
    cfg = STATE_CONFIGS["be_small"]
    n = cfg.n_cells
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, n), dtype=torch.int32, device=dev)
    opts = default_options(method=method, dt=2e-5, n_steps=100, form=CHEM_PERSISTENT)
    gm.chem_autotune(n, n, y0, None, opts)
    best = 1e30
    for _ in range(3):
        y.copy_(y0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - a)
    steps = int(cnt[0].sum().item())
    newton = int(cnt[2].sum().item())
    failed = int((st != 0).sum().item())
    it = counts.sdirk_iteration()
    # the guess S(y_n) once per step begun (completed steps plus a failed cell's last), the stage
    # bases and y_{n+1} once per completed step
    flops = (it.flops * newton + counts.sdirk_step_combination(stages).flops * steps
             + counts.source().flops * (steps + failed))
    r = {"workload": f"h2like_10_27, {n} cells, T0~U[1000,1500] K, Dirichlet(1), {label} 100 x 2e-7 s, persistent",
         "ms": best * 1e3, "cell_substeps_per_s": steps / best, "newton_iterations": newton,
         "flops_per_newton_iteration": it.flops, "tflops_algorithmic": flops / best / 1e12,
         "failed_cells": failed, "launch": list(gm.chem_get_launch(method, CHEM_PERSISTENT))}
    log(f"{label} 1024 cells: {best * 1e3:.2f} ms, {steps / best:.3e} cell-substeps/s, {newton} Newton iterations, "
        f"{flops / best / 1e12:.2f} TFLOP/s algorithmic, failed cells {r['failed_cells']}")
    return r


def yass_small_rate(gm, counts, solver, torch, np, dev, default_options, sample_states, STATE_CONFIGS):
    """YASS (Appendix A.4) on the 1,024-cell workload's states over its 2e-5 s at the paper's YASS
    step (200 steps of 1e-7 s, Table 5), LU or Jacobi-preconditioned GMRES (Section 3.4), persistent
    form, autotuned launch.  The algorithmic flop count is given for the LU solve (per attempt:
    Jacobian, source, LU and one solve, plus forming I - hJ and the decrement test)."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_YASS
    label = "LU" if solver == 0 else "GMRES (Jacobi)"
    cfg = STATE_CONFIGS["be_small"]
    n = cfg.n_cells
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, n), dtype=torch.int32, device=dev)
    opts = default_options(method=CHEM_YASS, dt=2e-5, n_steps=200, form=CHEM_PERSISTENT, linear_solver=solver)
    gm.chem_autotune(n, n, y0, None, opts)
    best = 1e30
    for _ in range(3):
        y.copy_(y0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - a)
    acc = int(cnt[0].sum().item())
    rej = int(cnt[1].sum().item())
    kry = int(cnt[2].sum().item())
    r = {"workload": f"h2like_10_27, {n} cells, T0~U[1000,1500] K, Dirichlet(1), YASS 200 x 1e-7 s, {label}, "
                     "alpha 0.1, persistent",
         "ms": best * 1e3, "cell_substeps_per_s": acc / best, "accepted_substeps": acc, "rejected_attempts": rej,
         "krylov_iterations": kry, "failed_cells": int((st != 0).sum().item()),
         "launch": list(gm.chem_get_launch(CHEM_YASS, CHEM_PERSISTENT))}
    if solver == 0:
        na = counts.na
        per = counts.jacobian(reduced=True) + counts.source() + counts.lu() + counts.solve()
        flops = (per.flops + na * na + 2 * na + 3 * na) * (acc + rej)
        r["tflops_algorithmic"] = flops / best / 1e12
    log(f"YASS {label} 1024 cells: {best * 1e3:.2f} ms, {acc / best:.3e} accepted substeps/s, {rej} rejections, "
        f"{kry} Krylov iterations, failed cells {r['failed_cells']}")
    return r


def be_small_rate(gm, torch, np, dev, default_options, CHEM_BE, sample_states, STATE_CONFIGS):
    """The 1,024-cell backward-Euler workload (200 steps of 1e-7 s, persistent form): a batch far
    too small to fill the GPU, reported for completeness."""
    cfg = STATE_CONFIGS["be_small"]
    n = cfg.n_cells
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, n), dtype=torch.int32, device=dev)
    opts = default_options(method=CHEM_BE, dt=2e-5, n_steps=200)
    best = 1e30
    for _ in range(3):
        y.copy_(y0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        gm.chem_integrate(n, n, y, None, opts, None, st, cnt)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - a)
    steps = int(cnt[0].sum().item())
    r = {"workload": f"h2like_10_27, {n} cells, T0~U[1000,1500] K, Dirichlet(1), backward Euler 200 x 1e-7 s, persistent",
         "ms": best * 1e3, "cell_substeps_per_s": steps / best, "newton_iterations": int(cnt[2].sum().item()),
         "failed_cells": int((st != 0).sum().item())}
    log(f"BE 1024 cells: {best * 1e3:.2f} ms, {steps / best:.3e} cell-substeps/s")
    return r


def adjoint_ratio(gm, torch, np, dev, Tape, default_options, CHEM_BE, sample_states, loss_weights, STATE_CONFIGS,
                  mech_name="h2like_10_27", T_range=(1000.0, 1500.0), alpha=1.0, reps=2):
    """Backward-Euler forward (with tape) vs discrete adjoint on the adjoint workload's 16,384
    cells (seed 2003): 500 x 2e-8 s steps, checkpoints every 50, dL/dy_N = w ~ N(0, 1).  Each time
    is the best of `reps` runs after one untimed forward + adjoint."""
    cfg = STATE_CONFIGS["adjoint_methane"]
    n = cfg.n_cells
    T, p, Y = sample_states(gm.ns, n, cfg.seed, T_range, alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, n), dtype=torch.int32, device=dev)
    opts = default_options(method=CHEM_BE, dt=1e-5, n_steps=500)
    tape = Tape(gm, n, 50)
    lam = t(np.ascontiguousarray(loss_weights(n, gm.n).T))
    d0 = torch.empty_like(y0)
    g = torch.zeros(gm.nr, dtype=torch.float64, device=dev)

    def timed(fn):
        torch.cuda.synchronize()
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - a

    def fwd(tp):
        y.copy_(y0)
        gm.chem_integrate(n, n, y, None, opts, tp, st, cnt)

    log(f"adjoint ({mech_name}): untimed forward + adjoint")
    fwd(tape)
    gm.chem_integrate_adjoint(tape, None, lam, d0, g)
    t_fwd = min(timed(lambda: fwd(None)) for _ in range(reps))
    t_fwd_tape = min(timed(lambda: fwd(tape)) for _ in range(reps))
    t_adj = min(timed(lambda: gm.chem_integrate_adjoint(tape, None, lam, d0, g)) for _ in range(reps))
    r = {"workload": f"{mech_name}, {n} cells, T0~U[{T_range[0]:.0f},{T_range[1]:.0f}] K, Dirichlet({alpha:g}), "
                     "backward Euler 500 x 2e-8 s, checkpoints every 50",
         "forward_ms": t_fwd * 1e3, "forward_with_tape_ms": t_fwd_tape * 1e3, "adjoint_ms": t_adj * 1e3,
         "adjoint_over_forward": t_adj / t_fwd, "total_over_forward": (t_fwd_tape + t_adj) / t_fwd,
         "newton_iterations": int(cnt[2].sum().item()), "failed_cells": int((st != 0).sum().item())}
    log(f"adjoint ({mech_name}): forward {t_fwd * 1e3:.1f} ms, with tape {t_fwd_tape * 1e3:.1f} ms, "
        f"adjoint {t_adj * 1e3:.1f} ms, ratio {t_adj / t_fwd:.2f}")
    return r


def ros2_adjoint_ratio(gm, torch, np, dev, Tape, default_options, sample_states, loss_weights, cfg, n=16384,
                       dt=1e-6, ckpt=50, max_steps=20000):
    """Rosenbrock forward (adaptive, persistent; with and without the tape) vs its discrete adjoint
    on the first n cells of the headline state distribution over the same split step."""
    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    y = torch.empty_like(y0)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, n), dtype=torch.int32, device=dev)
    opts = default_options(method=CHEM_ROS2, dt=dt, n_steps=0, form=CHEM_PERSISTENT)
    tape = Tape(gm, n, ckpt, method=CHEM_ROS2, max_steps=max_steps)
    lam = t(np.ascontiguousarray(loss_weights(n, gm.n).T))
    d0 = torch.empty_like(y0)
    g = torch.zeros(gm.nr, dtype=torch.float64, device=dev)

    def timed(fn):
        torch.cuda.synchronize()
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - a

    def fwd(tp):
        y.copy_(y0)
        gm.chem_integrate(n, n, y, None, opts, tp, st, cnt)

    fwd(tape)
    gm.chem_integrate_adjoint(tape, None, lam, d0, g)
    t_fwd = min(timed(lambda: fwd(None)) for _ in range(2))
    t_fwd_tape = min(timed(lambda: fwd(tape)) for _ in range(2))
    t_adj = min(timed(lambda: gm.chem_integrate_adjoint(tape, None, lam, d0, g)) for _ in range(2))
    acc = int(cnt[0].sum().item())
    r = {"workload": f"{gm.ns}-species mechanism, {n} cells of the headline state set, adaptive Rosenbrock over "
                     f"{dt:g} s, checkpoints every {ckpt} accepted steps",
         "forward_ms": t_fwd * 1e3, "forward_with_tape_ms": t_fwd_tape * 1e3, "adjoint_ms": t_adj * 1e3,
         "adjoint_over_forward": t_adj / t_fwd, "total_over_forward": (t_fwd_tape + t_adj) / t_fwd,
         "accepted_steps": acc, "max_accepted_per_cell": int(cnt[0].max().item()),
         "adjoint_steps_per_s": acc / t_adj, "failed_cells": int((st != 0).sum().item())}
    log(f"Rosenbrock adjoint: forward {t_fwd * 1e3:.1f} ms, with tape {t_fwd_tape * 1e3:.1f} ms, adjoint "
        f"{t_adj * 1e3:.1f} ms ({acc} accepted steps, max {r['max_accepted_per_cell']} per cell), ratio "
        f"{t_adj / t_fwd:.2f}, failed cells {r['failed_cells']}")
    return r


def large_mechanism_legs(torch, np, dev, args):
    """The 53-species / 325-reaction mechanism: its API kernels over the 262,144-cell state set and
    the adaptive Rosenbrock integration of args.c2_cells cells of that distribution over 1e-5 s
    (block form, persistent work queue with the probe/resume schedule, autotuned grid), with parity
    on the oracle's stored samples when the cell count is the samples' (4,096); the 150-species
    mechanism's API kernels."""
    import json as _json

    from paper_2510_10005_amd import CHEM_PERSISTENT, CHEM_ROS2, Mechanism, default_options
    from paper_2510_10005_amd.flops import MechanismCounts
    from synth import mechanism_file
    from synth.states import STATE_CONFIGS, sample_config, sample_states
    path = mechanism_file("ch4like_53_325")
    gm = Mechanism(path, KERNEL_CACHE)
    counts = MechanismCounts(path)
    cfg = STATE_CONFIGS["ros2_methane"]
    n = cfg.n_cells
    T, p, Y = sample_states(gm.ns, n, cfg.seed, cfg.T_range, cfg.alpha, cfg.p)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    y0 = torch.empty((gm.n, n), dtype=torch.float64, device=dev)
    gm.chem_state_from_TPY(n, n, t(T), t(p), t(Y.T), y0)
    out = {"workload": f"ch4like_53_325, {n} cells (seed {cfg.seed}), T0~U[800,2600] K, Dirichlet(0.5); source "
                       "terms one cell per lane, Jacobian one wavefront per cell"}
    out["api_kernels"] = api_kernel_rates(gm, counts, y0, n, torch, dev, reps=3)
    # adaptive Rosenbrock over the split step on nc cells of the set's distribution and seed (for
    # nc < 262,144 these are sample_config's nc cells, not a prefix of the full set)
    nc = max(1, min(args.c2_cells, n))
    if nc == n:
        y = y0.clone()
    else:
        Tc, pc, Yc = sample_config("ros2_methane", gm.ns, nc)
        y = torch.empty((gm.n, nc), dtype=torch.float64, device=dev)
        gm.chem_state_from_TPY(nc, nc, t(Tc), t(pc), t(Yc.T), y)
    yi = y.clone()
    st = torch.empty(nc, dtype=torch.int32, device=dev)
    cnt = torch.zeros((3, nc), dtype=torch.int32, device=dev)
    opts = default_options(method=CHEM_ROS2, dt=1e-5, n_steps=0, rtol=1e-6, atol=1e-10, form=CHEM_PERSISTENT)
    nt = min(nc, 1024)
    log(f"53-species Rosenbrock: autotuning on {nt} cells")
    gm.chem_autotune(nt, nc, yi, None, opts)
    block, grid = gm.chem_get_launch(CHEM_ROS2, CHEM_PERSISTENT)
    lus = gm.chem_get_lu_strategy(CHEM_ROS2)
    log(f"53-species Rosenbrock: {nc} cells over 1e-5 s, launch {block} x {grid}, LU strategy {lus}")
    # more than 32,768 cells: consecutive launches of 32,768 cells each (one line per launch)
    chunk = nc if nc <= 32768 else 32768
    wall = 0.0
    for c0 in range(0, nc, chunk):
        c1 = min(nc, c0 + chunk)
        yc = y[:, c0:c1].contiguous()
        stc = torch.empty(c1 - c0, dtype=torch.int32, device=dev)
        cc = torch.zeros((3, c1 - c0), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        a = time.perf_counter()
        gm.chem_integrate(c1 - c0, c1 - c0, yc, None, opts, None, stc, cc)
        torch.cuda.synchronize()
        dw = time.perf_counter() - a
        wall += dw
        y[:, c0:c1] = yc
        st[c0:c1] = stc
        cnt[:, c0:c1] = cc
        if chunk < nc:
            log(f"53-species Rosenbrock: cells {c0}..{c1 - 1} in {dw:.2f} s")
    acc = cnt[0].to(torch.float64)
    n_acc, n_rej = int(cnt[0].sum().item()), int(cnt[1].sum().item())
    att = counts.ros2_attempt()
    ros2 = {"workload": f"{nc} cells with the 262,144-cell set's distribution and seed, adaptive 2-stage Rosenbrock (rtol 1e-6, "
                        "atol 1e-10) over one 1e-5 s split step, block form (one cell per 256-thread workgroup), "
                        "persistent work queue, probe/resume schedule, autotuned grid",
            "cells": nc, "launch": {"block": block, "grid": grid, "cells_per_launch": chunk, "lu_strategy": lus},
            "ms": wall * 1e3,
            "accepted_substeps": n_acc, "rejected_attempts": n_rej,
            "cell_substeps_per_s": n_acc / wall, "attempts_per_s": (n_acc + n_rej) / wall,
            "substeps_min": int(acc.min().item()), "substeps_median": float(acc.median().item()),
            "substeps_max": int(acc.max().item()),
            "substep_max_over_min": float(acc.max().item() / max(1.0, acc.min().item())),
            "flops_per_attempt": att.flops,
            "tflops_algorithmic": att.flops * (n_acc + n_rej) / wall / 1e12,
            "failed_cells": int((st != 0).sum().item())}
    log(f"53-species Rosenbrock: {wall:.2f} s, {n_acc} accepted + {n_rej} rejected, {n_acc / wall:.3e} "
        f"cell-substeps/s, substeps per cell {ros2['substeps_min']}..{ros2['substeps_max']}")
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "ros2_methane_samples.json")
    if os.path.exists(gold):
        import oracle
        ref = _json.load(open(gold))
        om = oracle.load_mechanism(path)
        rows = [r for r in ref["cells"] if r["cell"] < nc] if nc == ref["subset"] else []
        if rows:
            idx = [r["cell"] for r in rows]
            yg = y[:, idx].cpu().numpy().T
            cg = cnt[:, idx].cpu().numpy()
            yo = np.array([r["y"] for r in rows])
            same = (cg[0] == np.array([r["accepted"] for r in rows])) & \
                   (cg[1] == np.array([r["rejected"] for r in rows]))
            # T relative; species as mass fractions relative to max(|Y_ref|, 1e-12)
            rho = (yo[:, 1:] * om.W).sum(axis=1)
            eT = np.abs(yg[:, 0] - yo[:, 0]) / np.abs(yo[:, 0])
            Yg, Yo = yg[:, 1:] * om.W / rho[:, None], yo[:, 1:] * om.W / rho[:, None]
            err = np.maximum(eT, (np.abs(Yg - Yo) / np.maximum(np.abs(Yo), 1e-12)).max(axis=1))
            ros2["parity"] = {"cells": len(idx), "cells_same_step_counts": int(same.sum()),
                              "max_rel_err": float(err.max()), "bar": 1e-8,
                              "reference": "oracle, stored per cell (tests/golden/ros2_methane_samples.json)"}
            log(f"53-species Rosenbrock parity: {int(same.sum())} of {len(idx)} sampled cells with equal step "
                f"counts, max rel err {err.max():.2e}")
    out["rosenbrock"] = ros2
    del y, yi, y0
    # 150-species mechanism: API kernels on the first 16,384 cells of its state set
    path150 = mechanism_file("large_150_1000")
    g150 = Mechanism(path150, KERNEL_CACHE)
    c150 = MechanismCounts(path150)
    cfg4 = STATE_CONFIGS["ros2_large"]
    n4 = 16384
    T4, p4, Y4 = sample_states(g150.ns, n4, cfg4.seed, cfg4.T_range, cfg4.alpha, cfg4.p)
    y4 = torch.empty((g150.n, n4), dtype=torch.float64, device=dev)
    g150.chem_state_from_TPY(n4, n4, t(T4), t(p4), t(Y4.T), y4)
    out["large_150_1000"] = {
        "workload": f"large_150_1000 (n = 151), first {n4} cells of its 65,536-cell set; source terms and "
                    "Jacobian in the block form (one cell per 256-thread workgroup)",
        "api_kernels": api_kernel_rates(g150, c150, y4, n4, torch, dev, reps=2),
        "integration": "not run: the integrators of this mechanism (factors in device memory) are off on the GPU "
                       "after an illegal memory access whose cause has not been shown"}
    return out


def _oracle_chunk(job):
    """One worker of the CPU baseline: the oracle's Rosenbrock integration of a chunk of cells with
    its BLAS limited to one thread."""
    mech_path, y0, dt = job
    from threadpoolctl import threadpool_limits

    import oracle
    om = oracle.load_mechanism(mech_path)
    with threadpool_limits(1):
        a = time.perf_counter()
        r = oracle.integrate_ros2(om, y0, dt)
        wall = time.perf_counter() - a
    return r["y"], r["status"], r["accepted"], r["rejected"], wall


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(path, cells_per_core, cfg, T, p, Y, y_gpu, counters_gpu):
    """The CPU oracle, as it stands, on all host cores (at most 16, the box's share for one GPU):
    one process per core, each integrating a chunk of cells_per_core cells of the seeded oracle
    subset of the workload (seed 5000) over the full split step with one BLAS thread.  The rate is
    the subset's accepted substeps over the wall time of the pool; the subset's final states are
    compared with the GPU's (cells with equal step counts, integrated-state bar 1e-8)."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    from synth.states import oracle_subset
    om = oracle.load_mechanism(path)
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    idx = oracle_subset(cfg.n_cells)[:cores * cells_per_core]
    y0 = oracle.state_from_TPY(om, T[idx], p[idx], Y[idx])
    chunks = [y0[k * cells_per_core:(k + 1) * cells_per_core] for k in range(cores)]
    log(f"cpu oracle: {len(idx)} cells of the seed-5000 subset on {cores} processes")
    ctx = mp.get_context("spawn")
    a = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_chunk, [(path, c, 1e-6) for c in chunks])
    wall = time.perf_counter() - a
    yo = np.concatenate([r[0] for r in res])
    so = np.concatenate([r[1] for r in res])
    acc_o = np.concatenate([r[2] for r in res])
    rej_o = np.concatenate([r[3] for r in res])
    acc = int(acc_o.sum())
    # parity on the subset
    yg = y_gpu[:, idx].T
    cg = counters_gpu[:, idx]
    same = (cg[0] == acc_o) & (cg[1] == rej_o) & (so == 0)
    rho = (yo[:, 1:] * om.W).sum(axis=1)
    eT = np.abs(yg[:, 0] - yo[:, 0]) / np.abs(yo[:, 0])
    Yg = yg[:, 1:] * om.W / rho[:, None]
    Yo = yo[:, 1:] * om.W / rho[:, None]
    eY = (np.abs(Yg - Yo) / np.maximum(np.abs(Yo), 1e-12)).max(axis=1)
    err = np.maximum(eT, eY)
    max_err = float(err[same].max()) if same.any() else None
    log(f"cpu oracle: {acc} cell-substeps in {wall:.1f} s on {cores} processes; parity on {int(same.sum())} of "
        f"{len(idx)} cells with equal step counts: max rel err {max_err}")
    return {"value": acc / wall, "unit": "cell-substeps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(idx)} cells of the seeded oracle subset (seed 5000) of the same 1,048,576-cell "
                      f"workload, full 1e-6 s split step, {cells_per_core} cells per process on {cores} processes "
                      f"(NumPy FP64, one BLAS thread each): {acc} accepted substeps in {wall:.1f} s",
            "parity": {"cells": len(idx), "cells_same_step_counts": int(same.sum()),
                       "max_rel_err_same_steps": max_err, "bar": 1e-8}}


if __name__ == "__main__":
    main()
