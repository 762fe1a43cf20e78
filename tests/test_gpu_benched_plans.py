"""GPU parity of the exact plans the benchmark times, on whole states.

Every plan here is built by bench.py's own plan functions (the same circuit,
k, flags and autotuner), specialised the way the benchmark specialises it, and
compared with the complex128 oracle computed in the test:

* the 28-qubit brickwork at k = 10 (tile tuned for specialised kernels, and
  at the 4 x 512 shape explicitly), its table-driven and gate-by-gate runs:
  all 2^28 amplitudes;
* the 32-qubit circuit's generator at 24 qubits, with the autotuned plan and
  with k = 10 at 4 x 512: all amplitudes and <sum Z_i Z_i+1>;
* the 20-qubit ansatz gradient plan (tuned tile and the shapes the tuner
  chooses from): energy and all 400 gradient entries against the oracle's
  adjoint, five against central differences of the oracle energy;
* the 2048-instance batched plan: energy, gradient and final state of
  sampled instances, for the three launch kinds the benchmark times.

Tolerances: max |amplitude error| <= 1e-5 (the target); relative l2 error
<= 8 u sqrt(G) with u = 2^-24 the float32 unit roundoff and G the gates
applied (rounding errors of independent gates add like a random walk, with
a few roundings per amplitude per gate); 1 - fidelity <= 1e-9 (of order the
square of the relative error).  Gradients within 1e-4 of the oracle.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2509_14098_amd as Q
import workloads as W

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402  (the benchmark's plan builders)

pytestmark = pytest.mark.gpu
TOL = 1e-5
U32 = 2.0 ** -24


def rel_bound(n_gates):
    return 8 * U32 * np.sqrt(n_gates)


@pytest.fixture(scope="module")
def sim():
    s = Q.Simulator(0)
    yield s
    s.close()


def whole_state_errors(psi, ref, chunk=1 << 24):
    """max-abs, relative l2 and 1 - fidelity over every amplitude (chunked
    device-to-host copies, float64 sums)."""
    m, d2, r2, g2, ov = 0.0, 0.0, 0.0, 0.0, 0j
    for i in range(0, ref.size, chunk):
        g = psi[i:i + chunk].cpu().numpy().astype(np.complex128)
        r = ref[i:i + chunk]
        d = g - r
        m = max(m, float(np.max(np.abs(d))))
        d2 += float(np.vdot(d, d).real)
        r2 += float(np.vdot(r, r).real)
        g2 += float(np.vdot(g, g).real)
        ov += complex(np.vdot(r, g))
    return m, np.sqrt(d2 / r2), 1 - abs(ov) ** 2 / (r2 * g2)


def check_state(psi, ref, n_gates, what):
    m, rel, inf = whole_state_errors(psi, ref)
    print(f"{what}: max-abs {m:.3e} rel-l2 {rel:.3e} 1-F {inf:.3e}", flush=True)
    assert m <= TOL, (what, m)
    assert rel <= rel_bound(n_gates), (what, rel)
    assert inf <= 1e-9, (what, inf)


# ---------------------------------------------------------------- 28-qubit headline

@pytest.fixture(scope="module")
def c2_ref():
    gates = W.brickwork_c2()
    return gates, oracle.apply(28, gates)


def _apply(sim, plan, n):
    psi = sim.zero_state(n)
    sim.apply(plan, psi)
    torch.cuda.synchronize()
    return psi


@pytest.mark.timeout(900)  # the first test also waits for the oracle's 28-qubit state
def test_headline_plan_tuned_and_specialised(sim, c2_ref):
    """The benchmark's headline plan: k = 10, tile tuned for specialised
    kernels, table-driven first, then one specialised kernel per partition."""
    gates, ref = c2_ref
    plan = bench.headline_plan(sim, 10)
    try:
        info = plan.info
        assert info["k_local"] == 10 and info["tile_qubits"] <= 13
        psi = _apply(sim, plan, 28)
        check_state(psi, ref, len(gates), f"C2 table-driven {info['reg_qubits']}x{1 << info['log_threads']}")
        sim.specialise(plan)
        psi = _apply(sim, plan, 28)
        check_state(psi, ref, len(gates), f"C2 specialised {info['reg_qubits']}x{1 << info['log_threads']}")
        z0 = float(sim.expect(W.z_on(0), psi, 28)[0])
        assert abs(z0 - oracle.expect(28, W.z_on(0), ref)) < 1e-5
    finally:
        plan.close()
    del psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tile", [(4, 9), (4, 8)])
def test_headline_plan_fixed_tiles_specialised(sim, c2_ref, tile):
    """k = 10 at the 13-qubit tile the tuner chose in earlier runs (4 x 512)
    and at the default 12-qubit tile, specialised."""
    gates, ref = c2_ref
    plan = bench.headline_plan(sim, 10, tile)
    try:
        assert (plan.info["reg_qubits"], plan.info["log_threads"]) == tile
        sim.specialise(plan)
        psi = _apply(sim, plan, 28)
        check_state(psi, ref, len(gates), f"C2 specialised tile {tile}")
    finally:
        plan.close()
    del psi
    torch.cuda.empty_cache()


def test_headline_gate_by_gate(sim, c2_ref):
    """The unfused baseline the benchmark times: one sweep per gate."""
    gates, ref = c2_ref
    plan = sim.partition(28, gates, 10, Q.PLAN_GATE_BY_GATE)
    try:
        assert plan.info["n_partitions"] == len(gates)
        psi = _apply(sim, plan, 28)
        check_state(psi, ref, len(gates), "C2 gate by gate")
    finally:
        plan.close()
    del psi
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- 32-qubit generator at 24 qubits

@pytest.fixture(scope="module")
def c3n24_ref():
    gates = W.brickwork_c3(n=24)
    return gates, oracle.apply(24, gates)


@pytest.mark.timeout(600)
def test_c3_generator_autotuned_plan(sim, c3n24_ref):
    """The benchmark's C3 flow (k and tile chosen by timing specialised
    candidates, then specialised) on the same generator at 24 qubits."""
    gates, ref = c3n24_ref
    plan, g = bench.c3_plan(sim, 24)
    try:
        assert np.array_equal(g, gates)
        sim.specialise(plan)
        psi = _apply(sim, plan, 24)
        info = plan.info
        check_state(psi, ref, len(gates), f"C3n24 tuned k={info['k_local']} {info['reg_qubits']}x"
                                          f"{1 << info['log_threads']}")
        zz = float(sim.expect(W.zz_chain(24), psi, 24)[0])
        assert abs(zz - oracle.expect(24, W.zz_chain(24), ref)) < 1e-5
    finally:
        plan.close()


def test_c3_generator_k10_tile_4x512(sim, c3n24_ref):
    """k = 10 at 4 x 512 (the shape the 32-qubit run was tuned to),
    table-driven and specialised."""
    gates, ref = c3n24_ref
    plan = sim.partition(24, gates, 10, 0, (4, 9))
    try:
        psi = _apply(sim, plan, 24)
        check_state(psi, ref, len(gates), "C3n24 k=10 4x512 table-driven")
        sim.specialise(plan)
        psi = _apply(sim, plan, 24)
        check_state(psi, ref, len(gates), "C3n24 k=10 4x512 specialised")
    finally:
        plan.close()


# ---------------------------------------------------------------- 20-qubit ansatz gradient

@pytest.fixture(scope="module")
def c4_ref():
    gates, npar = W.ansatz(20, 10)
    theta = W.ansatz_params(npar, seed=4)
    H = W.zz_chain_plus_x(20, 0.5)
    e, g = oracle.adjoint(20, gates, theta, H)
    return gates, theta, H, e, g


def _gradient(sim, plan, theta, H):
    psi = sim.zero_state(20)
    ckpt = sim.checkpoints(plan)
    sim.apply(plan, psi, theta, ckpt)
    e_fwd = float(sim.expect(H, psi, 20)[0])
    e, g = sim.adjoint_grad(plan, H, theta, psi, ckpt)
    torch.cuda.synchronize()
    return e_fwd, float(e[0]), g.cpu().numpy()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tile", [None, (3, 8), (4, 8), (5, 8)], ids=["tuned", "3x256", "4x256", "5x256"])
def test_c4_gradient_plan_specialised(sim, c4_ref, tile):
    """The benchmark's gradient plan (tile tuned for specialised kernels) and
    each fixed shape, specialised: forward sweeps and, for tiles of at most
    12 qubits, the generated reverse walk."""
    gates, theta, H, e_ref, g_ref = c4_ref
    plan, g2, th2, _ = bench.gradient_plan(sim, True, tile)
    try:
        assert np.array_equal(g2, gates) and np.array_equal(th2, theta)
        sim.specialise(plan)
        assert plan.info["specialised"] == 1
        e_fwd, e, g = _gradient(sim, plan, theta, H)
    finally:
        plan.close()
    err = float(np.max(np.abs(g - g_ref)))
    print(f"C4 tile {tile}: energy error {abs(e - e_ref):.2e}, gradient max error {err:.2e}", flush=True)
    assert abs(e_fwd - e_ref) < 1e-5 and abs(e - e_ref) < 1e-5
    assert err < 1e-4
    if tile is None:  # the benchmarked plan: also against central differences of the oracle energy
        h = 1e-3
        for j in (0, 1, 57, 200, 399):
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            fd = (oracle.expect(20, H, oracle.apply(20, gates, tp)) -
                  oracle.expect(20, H, oracle.apply(20, gates, tm))) / (2 * h)
            assert abs(g[j] - fd) < 1e-4, j


# ---------------------------------------------------------------- 2048 x 14-qubit batch

@pytest.mark.timeout(600)
def test_batched_plan_sampled_instances(sim):
    """The benchmark's batched plan: all 2048 instances in each of the three
    launches it times (forward; gradient from the forward's final states;
    forward + energy + gradient in one launch); energy, gradient and final
    state of 96 sampled instances (the first 64 and 32 more) against the
    oracle on each instance alone."""
    plan, circs, thetas, H = bench.batched_plan(sim)
    B, n = len(circs), 14
    theta = torch.as_tensor(np.concatenate(thetas), device="cuda")
    try:
        psi = torch.empty((B, 1 << n), dtype=torch.complex64, device="cuda")
        Q.qsv_apply(sim.ctx, plan.handle, theta, psi)
        e1, g1 = sim.adjoint_grad(plan, H, theta, psi)
        e2, g2 = sim.adjoint_grad(plan, H, theta)
        torch.cuda.synchronize()
    finally:
        plan.close()
    e1, g1, e2, g2 = (t.cpu().numpy() for t in (e1, g1, e2, g2))
    assert np.array_equal(e1, e2) and np.array_equal(g1, g2)
    offs = np.concatenate([[0], np.cumsum([len(t) for t in thetas])])
    sample = list(range(64)) + list(np.random.default_rng(77).choice(np.arange(64, B), 32, replace=False))
    worst_e = worst_g = worst_s = 0.0
    for b in sample:
        e_ref, g_ref = oracle.adjoint(n, circs[b], thetas[b], H)
        worst_e = max(worst_e, abs(e1[b] - e_ref))
        worst_g = max(worst_g, float(np.max(np.abs(g1[offs[b]:offs[b + 1]] - g_ref))))
        ref = oracle.apply(n, circs[b], thetas[b])
        worst_s = max(worst_s, float(np.max(np.abs(psi[b].cpu().numpy() - ref))))
    print(f"C5 96 instances: energy {worst_e:.2e} gradient {worst_g:.2e} state {worst_s:.2e}", flush=True)
    assert worst_e < 1e-5 and worst_g < 1e-4 and worst_s < TOL
