"""Benchmark of the partitioned state-vector hot path on one MI355X.

Headline (the `value`): the 28-qubit random brickwork circuit (40 layers of U3
on every qubit + alternating CZ/CX nearest-neighbour pairs + 5% random
long-range CX, seed 2, complex64, 2 GiB state), partitioned with k = 10 local
qubits, every partition running as its own specialised kernel (generated and
compiled before the timed region; the compile time is reported).  The tile
shape is chosen by the autotuner timing specialised candidates at k = 10.  One step =
the whole fused circuit applied to the state resident in HBM (every partition
sweep) plus <Z_0> reduced in float64.  value = algorithmic HBM bytes of the
step (16 B per amplitude per sweep + 8 B per amplitude for the expectation) /
step time, in GB/s.

Side measurements (separate timed regions, not in `value`):
  * the same plan on the table-driven sweep kernel (before specialising);
  * the same circuit gate by gate (one sweep per gate) -> fused speed-up;
  * the 28-qubit QFT (diagonal-heavy), fused and gate by gate;
  * the headline circuit with the distributed level (4 and 16 emulated ranks,
    remaps as SWAP sweeps);
  * the 32-qubit, 60-layer U3 + random-matching CX circuit with k and the tile
    shape chosen by the autotuner (timing specialised candidates), plus
    <sum Z_i Z_i+1>;
  * host planning time for 34-qubit circuits of 20 400 and 51 000 gates;
  * the 20-qubit RY.RZ + CX-ladder ansatz (400 parameters): adjoint gradient
    time / forward time (forward = apply + energy), specialised and
    table-driven;
  * 2048 x 14-qubit ansatz instances (depths 4..16): energy + gradient of all
    instances in one persistent launch;
  * the oracle (plain complex128 CPU simulator) on a bounded prefix of the
    headline circuit -> cpu_baseline.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

import paper_2509_14098_amd as Q
import workloads as W

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK = 157.3     # TFLOP/s (packed FP32 VALU; unpacked issue gives half)
FP32_UNPACKED_PEAK = 78.65   # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, without packed FP32
# Algorithmic flops per amplitude of one gate (the unfused gate list): a dense
# complex 2x2 takes 8 multiply-adds per output amplitude (16), a real rotation
# 8, a diagonal one complex multiply (6); permutations and sign flips none.
ALG_FLOPS = {"U3": 16, "RY": 8, "RZ": 6, "RX": 8, "H": 8, "CX": 0, "CZ": 0}


def algorithmic_flops(gates, n):
    """Flops of the gate list applied once to 2^n amplitudes, at ALG_FLOPS."""
    names = [W.KIND_NAME[int(k)] for k in gates["kind"]]
    missing = sorted(set(names) - set(ALG_FLOPS))
    if missing:
        raise ValueError(f"no algorithmic flop count for {missing}")
    return float(sum(ALG_FLOPS[x] for x in names)) * (1 << n)
HERE = os.path.dirname(os.path.abspath(__file__))
# HBM traffic of the headline's sweep kernels measured with rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE) on this workload, and the same counters for a plain
# 2 GiB copy: one summary per kernel kind, each for the tile shape it was taken on
TRAFFIC = {
    "specialised": (os.path.join(HERE, "profiles", "sweep_spec_traffic_c2_28q.txt"),
                    ["specialise.cpp", "rtc_options.h", "spec.cuh", "tile.cuh", "gates.cuh", "plan.h"]),
    "table-driven": (os.path.join(HERE, "profiles", "sweep_kernel_traffic_c2_28q.txt"),
                     ["sweep.hip", "tile.cuh", "gates.cuh", "plan.h"]),
}
# sources hashed by --copy-calibration's report (the specialised kernels')
SWEEP_SOURCES = TRAFFIC["specialised"][1]


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "paper_2509_14098_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sweep_sources_sha256():
    return sources_sha256(SWEEP_SOURCES)


def measured_traffic(kind="specialised", reg_qubits=4, log_threads=9):
    """HBM bytes per sweep launch from the committed counter summary of this
    kernel kind, scaled by the copy calibration; None if it is missing, was
    taken on other kernel sources or on another tile shape."""
    path, files = TRAFFIC[kind]
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sources_sha256") != sources_sha256(files):
            return None
        if (int(kv["reg_qubits"]), int(kv["log_threads"])) != (reg_qubits, log_threads):
            return None
        copy_bytes = float(kv["copy_bytes"])
        fetch = float(kv["sweep_fetch_kib_per_dispatch"]) * copy_bytes / float(kv["copy_fetch_kib_per_dispatch"])
        write = float(kv["sweep_write_kib_per_dispatch"]) * copy_bytes / float(kv["copy_write_kib_per_dispatch"])
        return fetch + write
    except (OSError, KeyError, ValueError):
        return None


def sync():
    torch.cuda.synchronize()


# The plans the benchmark times.  The parity tests build their plans through
# these same functions, so every benchmarked plan is also a tested plan.

def headline_plan(sim, k=10, tile=None, tune_specialised=True):
    """The 28-qubit brickwork at k local qubits; without a tile shape the
    autotuner picks one by timing specialised candidates at that k."""
    flags = Q.PLAN_TUNE_SPECIALISED if (tune_specialised and tile is None) else 0
    return sim.partition(28, W.brickwork_c2(), k, flags, tile)


def gradient_plan(sim, tune_specialised=True, tile=None):
    """The 20-qubit RY.RZ + CX-ladder ansatz (10 layers, 400 parameters) at
    k = 10 with checkpoints; without a tile shape it is tuned for specialised
    kernels."""
    gates, npar = W.ansatz(20, 10)
    flags = Q.PLAN_GRAD | (Q.PLAN_TUNE_SPECIALISED if (tune_specialised and tile is None) else 0)
    return sim.partition(20, gates, 10, flags, tile), gates, W.ansatz_params(npar, seed=4), W.zz_chain_plus_x(20, 0.5)


def c3_plan(sim, n=32, tune_specialised=True):
    """The U3 + random-matching CX circuit (60 layers) with k and the tile
    shape chosen by the autotuner."""
    gates = W.brickwork_c3(n=n)
    return sim.partition(n, gates, 0, Q.PLAN_TUNE_SPECIALISED if tune_specialised else 0), gates


def batched_plan(sim, B=2048, n=14):
    """B instances of the n-qubit ansatz with depths U{4..16} (seed 5) in
    one gradient plan; returns the plan, the circuits and their parameters."""
    circs, _, thetas = W.ansatz_batch(B, n, 4, 16, seed=5)
    gates = np.concatenate(circs)
    off = np.concatenate([[0], np.cumsum([len(c) for c in circs])])
    plan = sim.partition(n, gates, 0, Q.PLAN_GRAD, None, circ_offsets=off)
    return plan, circs, thetas, W.zz_chain_plus_x(n, 0.5)


def maybe_specialise(sim, plan, args):
    """Specialise the plan unless --no-specialise; the host seconds, or None
    where it stays table-driven (not asked, or a tile above 13 qubits)."""
    if args.no_specialise:
        return None
    try:
        return round(sim.specialise(plan), 2)
    except Q.QsvError:
        return None


def fused_step(sim, plan, psi, Hz0, out):
    sim.apply(plan, psi)
    Q.qsv_expect(sim.ctx, Hz0, plan.n, 1, psi, out)


def timed_steps(sim, plan, psi, Hz0, out, warmup, steps):
    """warmup + timed fused steps; returns (wall ms per step, summed sweep
    kernel ms from HIP events, number of timed sweep launches)."""
    for _ in range(warmup):
        fused_step(sim, plan, psi, Hz0, out)
    sync()
    Q.qsv_set_timing(sim.ctx, True)
    kernel_ms, launches = 0.0, 0
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fused_step(sim, plan, psi, Hz0, out)
        ms, nl = Q.qsv_last_sweep_ms(sim.ctx)  # waits for this step's last sweep event
        kernel_ms += ms
        launches += nl
    sync()
    wall = time.perf_counter() - t0
    Q.qsv_set_timing(sim.ctx, False)
    return wall * 1e3 / steps, kernel_ms, launches


def golden_sample_errors(sim, plan, psi, n, gates, name="c2"):
    """One fresh apply of the plan from |0..0> (outside any timed region),
    compared with the oracle's stored amplitudes of this circuit at a seeded
    sample of indices (tests/golden, written by a script that runs only the
    oracle): max-abs and relative l2 error over the sample."""
    path = os.path.join(HERE, "tests", "golden", f"{name}.npz")
    try:
        d = np.load(path)
    except OSError:
        return None
    if d["circuit_sha256"].item().decode() != W.circuit_hash(gates, n):
        return None
    psi.zero_()
    psi[0] = 1.0
    sim.apply(plan, psi)
    sync()
    idx, ref = d["idx"], d["amp"]
    got = psi[torch.as_tensor(idx, device=psi.device)].cpu().numpy().astype(np.complex128)
    diff = got - ref
    return dict(sample=int(len(idx)), max_abs=float(np.max(np.abs(diff))),
                rel_l2=float(np.linalg.norm(diff) / np.linalg.norm(ref)), oracle="complex128, stored sample")


def bench_headline(sim, args):
    n, k = 28, args.k
    gates = W.brickwork_c2()
    tile = tuple(args.tile) if args.tile else None
    # the tile shape is tuned at k = 10 by timing specialised candidates (unless given)
    plan = headline_plan(sim, k, tile, not args.no_specialise)
    tuned = [list(c) for c in Q.qsv_last_autotune()] if not (args.no_specialise or tile) else None
    psi = sim.zero_state(n)
    Hz0 = W.z_on(0)
    out = torch.empty(1, dtype=torch.float64, device=sim.device)
    res = {}
    if not args.no_specialise:
        # the same plan on the table-driven sweep first, then specialised
        ms, kms, nl = timed_steps(sim, plan, psi, Hz0, out, 1, 3)
        res["table_driven"] = dict(ms_per_step=round(ms, 3), avg_launch_ms=round(kms / max(1, nl), 4))
        res["specialise_s"] = round(sim.specialise(plan), 2)
    step_ms, kernel_ms, launches = timed_steps(sim, plan, psi, Hz0, out, args.warmup, args.steps)
    info = plan.info
    dim = 1 << n
    step_bytes = info["bytes_per_apply"] + 8.0 * dim
    res.update(plan=info, step_ms=step_ms, step_bytes=step_bytes, kernel_ms_total=kernel_ms, launches=launches,
               z0=float(out[0]), tile_candidates=tuned, alg_flops=algorithmic_flops(gates, n))
    res["errors"] = golden_sample_errors(sim, plan, psi, n, gates)
    plan.close()
    # gate by gate: same kernels, one gate per partition
    if not args.skip_gbg:
        plan_g = sim.partition(n, gates, k, Q.PLAN_GATE_BY_GATE, tile)
        sim.apply(plan_g, psi)
        sync()
        t0 = time.perf_counter()
        sim.apply(plan_g, psi)
        sync()
        res["gbg_ms"] = (time.perf_counter() - t0) * 1e3
        res["gbg_sweeps"] = plan_g.info["n_partitions"]
        plan_g.close()
    del psi
    torch.cuda.empty_cache()
    return res


def bench_gradient(sim, args):
    n = 20
    # the tile shape is tuned at k = 10 by timing specialised candidates (unless not specialising)
    plan, gates, theta_np, H = gradient_plan(sim, not args.no_specialise)
    npar = len(theta_np)
    theta = torch.as_tensor(theta_np, device=sim.device)
    tile = [plan.info["reg_qubits"], plan.info["log_threads"]]
    psi = sim.zero_state(n)
    ckpt = sim.checkpoints(plan)
    out = torch.empty(1, dtype=torch.float64, device=sim.device)
    energy = torch.empty(1, dtype=torch.float64, device=sim.device)
    grad = torch.empty(npar, dtype=torch.float64, device=sim.device)

    def forward():
        psi.zero_()
        psi[0] = 1.0
        sim.apply(plan, psi, theta, ckpt)
        Q.qsv_expect(sim.ctx, H, n, 1, psi, out)

    def backward():
        Q.qsv_adjoint_grad(sim.ctx, plan.handle, H, theta, psi, ckpt, energy, grad)

    def timed():
        for _ in range(3):
            forward()
            backward()
        sync()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            forward()
        sync()
        t_fwd = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            backward()
        sync()
        t_bwd = (time.perf_counter() - t0) / reps
        return t_fwd * 1e3, t_bwd * 1e3

    # the table-driven kernels first, then the plan specialised (forward sweeps
    # and adjoint walk generated per partition)
    f0, b0 = timed()
    res = dict(fwd_ms=f0, grad_ms=b0, ratio=b0 / f0)
    spec_s = maybe_specialise(sim, plan, args)
    if spec_s is not None:
        f1, b1 = timed()
        res = dict(fwd_ms=f1, grad_ms=b1, ratio=b1 / f1, specialise_s=spec_s,
                   table_driven=dict(fwd_ms=round(f0, 4), grad_ms=round(b0, 4), ratio=round(b0 / f0, 4)))
    # the energy alone (qsv_expect of H on the forward's state: term upload,
    # tile passes, final sum), GPU time between events around each call
    for _ in range(3):
        Q.qsv_expect(sim.ctx, H, n, 1, psi, out)
    sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for e0, e1 in ev:
        e0.record()
        Q.qsv_expect(sim.ctx, H, n, 1, psi, out)
        e1.record()
    sync()
    res["energy_us"] = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])) * 1e3
    res.update(energy=float(energy[0]), partitions=plan.info["n_partitions"], tile=tile)
    res["_grad"] = grad.cpu().numpy()  # compared with the oracle in the CPU leg
    res["_energy"] = float(energy[0])
    plan.close()
    return res


def batched_timings(sim, plan, theta, H, B, n):
    """Forward (final states of every instance), adjoint from those states,
    and forward + energy + adjoint from |0>, each averaged over 5 calls; the
    load balance of one more forward and forward + energy + adjoint (each
    workgroup's exit on the device clock, from the first workgroup's start)."""
    energy = torch.empty(B, dtype=torch.float64, device=sim.device)
    grad = torch.empty(len(theta), dtype=torch.float64, device=sim.device)
    psi = torch.empty((B, 1 << n), dtype=torch.complex64, device=sim.device)
    reps = 5

    def timed(fn):
        for _ in range(2):
            fn()
        sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        sync()
        return (time.perf_counter() - t0) / reps

    dtf = timed(lambda: Q.qsv_apply(sim.ctx, plan.handle, theta, psi))
    dtg = timed(lambda: Q.qsv_adjoint_grad(sim.ctx, plan.handle, H, theta, psi, None, energy, grad))
    dt = timed(lambda: Q.qsv_adjoint_grad(sim.ctx, plan.handle, H, theta, None, None, energy, grad))
    balance = {}
    Q.qsv_set_timing(sim.ctx, True)
    for kind, fn in (("forward", lambda: Q.qsv_apply(sim.ctx, plan.handle, theta, psi)),
                     ("fwd_energy_grad", lambda: Q.qsv_adjoint_grad(sim.ctx, plan.handle, H, theta, None, None,
                                                                    energy, grad))):
        fn()
        clk, hz = Q.qsv_last_batch_clock(sim.ctx)
        if len(clk) and hz > 0:
            start = clk[:, 0].astype(np.float64).min()
            ends = (clk[:, 1].astype(np.float64) - start) / hz * 1e3
            balance[kind] = dict(workgroups=int(len(clk)), last_exit_ms=round(float(ends.max()), 3),
                                 mean_exit_ms=round(float(ends.mean()), 3), first_exit_ms=round(float(ends.min()), 3),
                                 tail_frac=round(float((ends.max() - ends.mean()) / ends.max()), 4))
    Q.qsv_set_timing(sim.ctx, False)
    return dtf, dtg, dt, balance, energy, grad


def start_batched_specialise(sim, B=2048, n=14):
    """The batched plan of bench_batched, its specialised kernel compiling in
    the background (helper process) while the other legs run."""
    plan, circs, thetas, H = batched_plan(sim, B, n)
    sim.specialise_async(plan)
    return plan, circs, thetas, H, time.perf_counter()


def bench_batched(sim, args, spec=None):
    """2048 instances of the 14-qubit ansatz (depths U{4..16}), energy and
    gradient of every instance.  Table-driven kernel, then (spec given) the
    plan whose kernel specialised for its 13 circuit structures was compiled
    in the background: its forward launches run specialised, the adjoint walk
    table-driven from the forward's final states."""
    n, B = 14, 2048
    t0 = time.perf_counter()
    plan, circs, thetas, H = batched_plan(sim, B, n)
    plan_s = time.perf_counter() - t0
    gates = np.concatenate(circs)
    theta = torch.as_tensor(np.concatenate(thetas), device=sim.device)
    dtf, dtg, dt, balance, energy, grad = batched_timings(sim, plan, theta, H, B, n)
    info = plan.info
    plan.close()
    fwd_flops = algorithmic_flops(gates, n)  # every instance's gate list on its 2^n amplitudes
    table = dict(forward_ms=round(dtf * 1e3, 3), grad_ms=round(dtg * 1e3, 3),
                 fwd_energy_grad_ms=round(dt * 1e3, 3), forward_frac_of_fp32_peak=round(
                     fwd_flops / dtf / 1e12 / FP32_VECTOR_PEAK, 4), load_balance=balance)
    kernel = "table-driven"
    spec_info = {}
    if spec is not None:
        splan, _, _, _, started = spec
        t1 = time.perf_counter()
        try:
            secs = sim.specialise(splan)  # waits for the background compile
        except Q.QsvError as e:  # the compile failed: the table-driven figures stand
            spec_info = dict(specialise_error=str(e)[:300])
            secs = None
        if secs is not None:
            spec_info = dict(specialise_s=round(secs, 2), waited_s=round(time.perf_counter() - t1, 2),
                             started_s_before=round(t1 - started, 2))
            dtf, dtg, dt, balance, energy, grad = batched_timings(sim, splan, theta, H, B, n)
            kernel = "specialised forward (one kernel, every circuit structure compiled in), table-driven adjoint"
        splan.close()
    offs = np.concatenate([[0], np.cumsum([len(t) for t in thetas])])
    n_check = 64  # instances compared with the oracle in the CPU leg
    e_np, g_np = energy.cpu().numpy(), grad.cpu().numpy()
    checked = dict(energy=e_np[:n_check], grad=[g_np[offs[b]:offs[b + 1]] for b in range(n_check)])
    res = dict(_checked=checked, instances=B, n_qubits=n, gates=int(len(gates)), params=int(len(theta)),
               kernel=kernel, load_balance=balance, forward_alg_tflops=round(fwd_flops / dtf / 1e12, 2),
               forward_frac_of_fp32_peak=round(fwd_flops / dtf / 1e12 / FP32_VECTOR_PEAK, 4),
               forward_ms=round(dtf * 1e3, 3), grad_ms=round(dtg * 1e3, 3), grad_over_forward=round(dtg / dtf, 3),
               fwd_energy_grad_ms=round(dt * 1e3, 3), fwd_energy_grad_over_forward=round(dt / dtf, 3),
               instances_per_s=round(B / dt, 1), register_stages=info["n_stages"], plan_seconds=round(plan_s, 3))
    if spec is not None:
        res.update(spec_info, table_driven=table)
    return res


def bench_qft(sim, args):
    """28-qubit textbook QFT (28 H, 378 controlled phases, 14 SWAP): a
    diagonal-heavy circuit, fused at k = 10 against gate by gate."""
    n = 28
    gates = W.qft(n)
    psi = sim.zero_state(n)
    res = dict(n_qubits=n, n_gates=int(len(gates)))
    for flags, key in ((0, "fused"), (Q.PLAN_GATE_BY_GATE, "gate_by_gate")):
        plan = sim.partition(n, gates, 10, flags, None)
        spec_s = maybe_specialise(sim, plan, args) if flags == 0 else None
        sim.apply(plan, psi)
        sync()
        t0 = time.perf_counter()
        sim.apply(plan, psi)
        sync()
        dt = time.perf_counter() - t0
        sweeps = plan.info["n_partitions"]
        res[key] = dict(ms=round(dt * 1e3, 2), sweeps=sweeps, gbs=round(16.0 * (1 << n) * sweeps / dt / 1e9, 1))
        if flags == 0:
            res[key]["specialise_s"] = spec_s
        plan.close()
    res["fused_speedup"] = round(res["gate_by_gate"]["ms"] / res["fused"]["ms"], 2)
    del psi
    torch.cuda.empty_cache()
    return res


def bench_distributed(sim, args):
    """The headline circuit and the 28-qubit QFT with the distributed level:
    2^g emulated ranks of 2^(28-g) amplitudes, remaps between distributed
    partitions done as SWAP sweeps on this GPU.  Each sweep is timed with HIP
    events, which splits the apply into local computation (compute sweeps)
    and data movement (remap sweeps)."""
    n = 28
    psi = sim.zero_state(n)
    res = {}
    for name, gates in (("c2", W.brickwork_c2()), ("qft", W.qft(n))):
        for g in (2, 4):
            plan = sim.partition_distributed(n, gates, g, args.k)
            spec_s = maybe_specialise(sim, plan, args)
            di = Q.qsv_plan_distributed_info(plan.handle)
            parts = plan.partitions()
            is_remap = [bool(gl) and gl[0] < 0 for _, gl in parts]
            sim.apply(plan, psi)
            sync()
            t0 = time.perf_counter()
            sim.apply(plan, psi)
            sync()
            dt = time.perf_counter() - t0
            Q.qsv_set_timing(sim.ctx, True)
            sim.apply(plan, psi)
            times = Q.qsv_last_sweep_times(sim.ctx)
            Q.qsv_set_timing(sim.ctx, False)
            remap_ms = float(sum(t for t, r in zip(times, is_remap) if r))
            res[f"{name}_g{g}"] = dict(
                ranks=1 << g, dist_partitions=di["n_dist_partitions"], exchange_swaps=di["exchange_swaps"],
                remap_swaps=di["remap_swaps"], sweeps=plan.info["n_partitions"], remap_sweeps=sum(is_remap),
                ms=round(dt * 1e3, 2), compute_sweeps_ms=round(float(sum(times)) - remap_ms, 2),
                remap_sweeps_ms=round(remap_ms, 2), specialise_s=spec_s)
            plan.close()
    del psi
    torch.cuda.empty_cache()
    return res


def bench_planner(args):
    """Host planning time of all three levels of the paper's memory hierarchy
    (distributed ranks of 28 local qubits, tiles of k = 10, register stages;
    contraction graph, closeness, greedy at each level, lowering; no device
    upload) on U3 + random-matching CX circuits of 30, 34 and 37 qubits with
    about 2*10^4 and 10^5 gates."""
    res = []
    for n, layers in ((30, 400), (34, 400), (37, 400), (30, 2200), (37, 2000)):
        gates = W.brickwork_c3(n=n, layers=layers, seed=7)
        g = n - 28
        t0 = time.perf_counter()
        plan = Q.qsv_partition_distributed(None, n, gates, g, args.k, 0, None)
        dt = time.perf_counter() - t0
        info = Q.qsv_plan_info(plan)
        di = Q.qsv_plan_distributed_info(plan)
        Q.qsv_plan_destroy(plan)
        res.append(dict(n_qubits=n, n_gates=int(len(gates)), ranks=1 << g, seconds=round(dt, 3),
                        dist_partitions=di["n_dist_partitions"], tile_partitions=info["n_partitions"],
                        register_stages=info["n_stages"]))
    return res


def bench_c3(sim, args):
    """32-qubit local share (60 layers of U3 + random CX matchings): the
    autotuner chooses k and the tile shape, then one apply and <sum Z_i Z_i+1>."""
    n = 32
    t0 = time.perf_counter()
    plan, gates = c3_plan(sim, n, not args.no_specialise)
    plan_s = time.perf_counter() - t0
    spec_s = maybe_specialise(sim, plan, args)
    info = plan.info
    psi = sim.zero_state(n)
    H = W.zz_chain(n)
    out = torch.empty(1, dtype=torch.float64, device=sim.device)
    sync()
    t0 = time.perf_counter()
    sim.apply(plan, psi)
    Q.qsv_expect(sim.ctx, H, n, 1, psi, out)
    sync()
    dt = time.perf_counter() - t0
    plan.close()
    del psi
    torch.cuda.empty_cache()
    return dict(n_qubits=n, n_gates=int(len(gates)), k_local=info["k_local"], reg_qubits=info["reg_qubits"],
                log_threads=info["log_threads"], partitions=info["n_partitions"],
                plan_and_tune_s=round(plan_s, 2), candidates=[list(c) for c in Q.qsv_last_autotune()],
                specialise_s=spec_s,
                apply_expect_ms=round(dt * 1e3, 1),
                gbs=round((info["bytes_per_apply"] + 8.0 * (1 << n)) / dt / 1e9, 1), zz=float(out[0]))


SINGLE_CORE_CHILD = r"""
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
import oracle, workloads as W
n, limit = 28, float(sys.argv[2])
gates = W.brickwork_c2()
psi = oracle.zero_state(n)
done, t = 0, 0.0
while done < len(gates) and t < limit:
    t0 = time.perf_counter()
    oracle.apply_range(n, gates, done, done + 1, psi)
    t += time.perf_counter() - t0
    done += 1
print(json.dumps(dict(gates=done, seconds=t, threads=oracle.threads(), cpus=sorted(os.sched_getaffinity(0)))))
"""


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_single_core(args, gpu_bytes_per_apply, n_gates_total):
    """The oracle pinned to one host core with one OpenMP thread (a child
    process, so the thread count is fixed before the OpenMP runtime starts)."""
    import subprocess
    cpu = min(os.sched_getaffinity(0))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", SINGLE_CORE_CHILD, HERE, str(args.cpu_seconds / 2)], env=env,
                       capture_output=True, text=True, timeout=600,
                       preexec_fn=lambda: os.sched_setaffinity(0, {cpu}))
    if r.returncode != 0:
        return dict(error=r.stderr[-500:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return dict(value=gpu_bytes_per_apply * d["gates"] / n_gates_total / d["seconds"] / 1e9, unit="GB/s",
                cores=1, threads=d["threads"], pinned_cpus=d["cpus"],
                sample=f"first {d['gates']} of {n_gates_total} gates of the 28-qubit headline circuit on one core, "
                       f"{d['seconds']:.1f} s")


def bench_one_shot(sim, args):
    """End-to-end time of one apply + <H> starting from the gate list (plan,
    then apply; state allocated beforehand) on the 28-qubit headline circuit and
    the 32-qubit circuit at k = 10 and the default tile: table-driven, and with
    the specialised kernels compiled in the background
    (qsv_plan_specialise_async) while the apply runs, each partition switching
    to its kernel once that is loaded.  The synchronous policy (tune, compile,
    then apply) is the sum of the headline's and the C3 leg's own figures."""
    res = {}
    for name, n, gates, H in (("c2", 28, W.brickwork_c2(), W.z_on(0)), ("c3", 32, W.brickwork_c3(), W.zz_chain(32))):
        psi = sim.zero_state(n)
        out = torch.empty(1, dtype=torch.float64, device=sim.device)
        r = {}
        for policy in ("table_driven", "async_specialise"):
            psi.zero_()
            psi[0] = 1.0
            sync()
            t0 = time.perf_counter()
            plan = sim.partition(n, gates, 10)  # the default tile, no tuning
            if policy != "table_driven":
                sim.specialise_async(plan)
            sim.apply(plan, psi)
            Q.qsv_expect(sim.ctx, H, n, 1, psi, out)
            sync()
            r[policy + "_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
            if policy != "table_driven":
                r["specialised_by_the_end"] = bool(plan.refresh()["specialised"])
            plan.close()  # joins a compile still running (outside the timed region)
        res[name] = r
        del psi
        torch.cuda.empty_cache()
    return res


def bench_oracle(args, gpu_bytes_per_apply, n_gates_total, gpu_results):
    """The oracle on a bounded prefix of the headline circuit (~10-30 s), on
    all host threads and pinned to one core; the oracle's 20-qubit gradient and
    64 of the 2048 batched instances, timed and compared with the GPU's."""
    import oracle
    n = 28
    gates = W.brickwork_c2()
    psi = oracle.zero_state(n)
    done, t_total = 0, 0.0
    chunk = 4
    while done < len(gates) and t_total < args.cpu_seconds:
        t0 = time.perf_counter()
        oracle.apply_range(n, gates, done, min(done + chunk, len(gates)), psi)
        t_total += time.perf_counter() - t0
        done = min(done + chunk, len(gates))
    del psi
    frac = done / n_gates_total
    res = dict(value=gpu_bytes_per_apply * frac / t_total / 1e9, unit="GB/s", cores=oracle.threads(), kind="oracle",
               sample=f"first {done} of {n_gates_total} gates of the 28-qubit headline circuit, complex128 gate by "
                      f"gate, {t_total:.1f} s; rate expressed as the fused circuit's algorithmic bytes x fraction "
                      f"of gates done / time",
               cpu_model=cpu_model(), circuit_sha256=W.circuit_hash(gates, n))
    res["single_core"] = oracle_single_core(args, gpu_bytes_per_apply, n_gates_total)
    errors = {}
    # the same oracle on the smaller workloads, in full or on a stated sample
    t0 = time.perf_counter()
    oracle.apply(12, W.brickwork_c1())
    res["c1_full_s"] = round(time.perf_counter() - t0, 4)
    g4, np4 = W.ansatz(20, 10)
    th4 = W.ansatz_params(np4, seed=4)
    H = W.zz_chain_plus_x(20, 0.5)
    t0 = time.perf_counter()
    oracle.apply(20, g4, th4)
    res["c4_forward_s"] = round(time.perf_counter() - t0, 3)
    t0 = time.perf_counter()
    e4, gr4 = oracle.adjoint(20, g4, th4, H)
    res["c4_energy_gradient_s"] = round(time.perf_counter() - t0, 3)
    adj = gpu_results.get("adjoint")
    if adj is not None:
        errors["c4_energy_abs"] = abs(adj["_energy"] - e4)
        errors["c4_grad_max_abs"] = float(np.max(np.abs(adj["_grad"] - gr4)))
    circs, _, thetas = W.ansatz_batch(2048, 14, 4, 16, seed=5)
    H14 = W.zz_chain_plus_x(14, 0.5)
    t0 = time.perf_counter()
    ref5 = [oracle.adjoint(14, circs[b], thetas[b], H14) for b in range(64)]
    res["c5_energy_gradient_instances_per_s"] = round(64 / (time.perf_counter() - t0), 1)
    res["c5_sample"] = "first 64 of the 2048 14-qubit instances"
    bat = gpu_results.get("batched")
    if bat is not None:
        chk = bat["_checked"]
        errors["c5_instances"] = len(ref5)
        errors["c5_energy_max_abs"] = float(max(abs(chk["energy"][b] - ref5[b][0]) for b in range(len(ref5))))
        errors["c5_grad_max_abs"] = float(max(np.max(np.abs(chk["grad"][b] - ref5[b][1])) for b in range(len(ref5))))
    return res, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--tile", type=int, nargs=2, default=None, help="reg_qubits log_threads")
    ap.add_argument("--no-specialise", action="store_true",
                    help="headline on the table-driven sweep kernel instead of per-partition kernels")
    ap.add_argument("--skip-gbg", action="store_true")
    ap.add_argument("--skip-grad", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-c3", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy 5 times (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        sync()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        sync()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps(dict(copy_bytes_read=8 << 28, copy_bytes_written=8 << 28, launches=10,
                              copy_gbs=round(2 * (8 << 28) / dt / 1e9, 1), sources_sha256=sweep_sources_sha256())))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU path is not part of this "
              f"build", file=sys.stderr)
        sys.exit(2)
    sim = Q.Simulator(0)
    # the batched plan's specialised kernel compiles in the background meanwhile
    bspec = None if args.skip_batched or args.no_specialise else start_batched_specialise(sim)
    head = bench_headline(sim, args)
    info = head["plan"]
    value = head["step_bytes"] / (head["step_ms"] * 1e-3) / 1e9
    avg_launch_ms = head["kernel_ms_total"] / max(1, head["launches"])
    sweep_bytes = 16.0 * (1 << 28)
    n_launch = info["n_partitions"]
    # roofline of the dominant kernels (the partition sweeps): algorithmic flops
    # of the gate list (U3 16, RY 8, RZ 6, RX 8, H 8, CX/CZ 0 per amplitude) per
    # launch, i.e. the circuit's total over its sweeps; the count the kernels
    # execute after diagonal folding is reported beside it
    alg_flops = head["alg_flops"] / n_launch
    exec_flops = info["flops_per_apply"] / n_launch
    intensity = alg_flops / sweep_bytes
    ridge = FP32_VECTOR_PEAK * 1e12 / (HBM_PEAK_GBS * 1e9)
    achieved_gbs = sweep_bytes / (avg_launch_ms * 1e-3) / 1e9
    achieved_tf = alg_flops / (avg_launch_ms * 1e-3) / 1e12
    exec_tf = exec_flops / (avg_launch_ms * 1e-3) / 1e12
    traffic = measured_traffic("specialised" if info["specialised"] else "table-driven", info["reg_qubits"],
                               info["log_threads"])
    traffic = None if traffic is None else round(traffic)
    if intensity > ridge:
        roof = dict(bound="alu", achieved=round(achieved_tf, 3), peak=FP32_VECTOR_PEAK, unit="TFLOP/s",
                    frac=round(achieved_tf / FP32_VECTOR_PEAK, 4), traffic=traffic)
    else:
        roof = dict(bound="hbm", achieved=round(achieved_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved_gbs / HBM_PEAK_GBS, 4), traffic=traffic)
    line = dict(
        metric="state-vector sweep GB/s (% HBM peak); adjoint grad time / forward; fused vs gate-by-gate",
        value=round(value, 2), unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(head["step_ms"], 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="c64/f32 (f64 reductions)", data="synthetic",
        config=dict(workload="28-qubit random brickwork, 40 layers, U3 + CZ/CX pairs + 5% long-range CX, seed 2, "
                             "complex64 2 GiB, k=10 fused sweeps + <Z0>",
                    n_qubits=28, n_gates=info["n_gates"], k_local=info["k_local"], tile_qubits=info["tile_qubits"],
                    reg_qubits=info["reg_qubits"], log_threads=info["log_threads"],
                    partitions=info["n_partitions"], register_stages=info["n_stages"],
                    plan_and_tune_seconds=round(info["plan_seconds"], 3),
                    tile_candidates=head.get("tile_candidates"),
                    kernels="one specialised kernel per partition" if info["specialised"] else "table-driven sweep",
                    specialise_seconds=head.get("specialise_s")),
        hbm_frac=round(value / HBM_PEAK_GBS, 4),
        roofline=roof,
        roofline_hbm=dict(achieved=round(achieved_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(achieved_gbs / HBM_PEAK_GBS, 4),
                          traffic_over_algorithmic=None if traffic is None else round(traffic / sweep_bytes, 4)),
        sweep=dict(avg_launch_ms=round(avg_launch_ms, 4), launches_per_step=n_launch, bytes_per_launch=sweep_bytes,
                   alg_flops_per_launch=alg_flops, alg_flops_per_byte=round(intensity, 2),
                   ridge_flops_per_byte=round(ridge, 2), alg_tflops=round(achieved_tf, 3),
                   executed_flops_per_launch=exec_flops, executed_tflops=round(exec_tf, 3),
                   executed_frac_of_unpacked_fp32=round(exec_tf / FP32_UNPACKED_PEAK, 4)),
        hbm_target=dict(target_frac=0.70, achieved_frac=round(achieved_gbs / HBM_PEAK_GBS, 4),
                        met=achieved_gbs / HBM_PEAK_GBS >= 0.70),
        errors=dict(c2_sample=head.get("errors")),
    )
    if "table_driven" in head:
        td = head["table_driven"]
        line["table_driven"] = dict(td, speedup_of_specialised=round(td["ms_per_step"] / head["step_ms"], 3))
    if "gbg_ms" in head:
        line["gate_by_gate"] = dict(ms=round(head["gbg_ms"], 2), sweeps=head["gbg_sweeps"],
                                    gbs=round(16.0 * (1 << 28) * head["gbg_sweeps"] / (head["gbg_ms"] * 1e-3) / 1e9, 1),
                                    # both sides are wall-clock times of whole applies (the fused step also
                                    # holds the <Z0> reduction)
                                    fused_speedup=round(head["gbg_ms"] / head["step_ms"], 2))
    if not args.skip_grad:
        line["adjoint"] = {k: (round(v, 4) if isinstance(v, float) and not k.startswith("_") else v)
                           for k, v in bench_gradient(sim, args).items()}
    if not args.skip_batched:
        line["batched"] = bench_batched(sim, args, bspec)
    if not args.skip_gbg:
        line["qft"] = bench_qft(sim, args)
        line["distributed"] = bench_distributed(sim, args)
    if not args.skip_c3:
        line["c3_autotuned"] = bench_c3(sim, args)
        line["planner"] = bench_planner(args)
        one = bench_one_shot(sim, args)
        c3 = line["c3_autotuned"]
        one["c2"]["tune_and_specialise_ms"] = round(
            (info["plan_seconds"] + (head.get("specialise_s") or 0)) * 1e3 + head["step_ms"], 1)
        one["c3"]["tune_and_specialise_ms"] = round(
            (c3["plan_and_tune_s"] + (c3["specialise_s"] or 0)) * 1e3 + c3["apply_expect_ms"], 1)
        line["one_shot"] = one
    sim.close()
    if not args.skip_cpu:
        line["cpu_baseline"], errs = bench_oracle(args, info["bytes_per_apply"], info["n_gates"], line)
        line["errors"].update(errs)
    else:
        line["cpu_baseline"] = None
    for key in ("adjoint", "batched"):  # arrays kept for the oracle comparison only
        for k in [k for k in line.get(key, {}) if k.startswith("_")]:
            del line[key][k]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
