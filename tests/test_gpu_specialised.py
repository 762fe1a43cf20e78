"""GPU parity of specialised plans (qsv_plan_specialise: one generated kernel
per partition, Section 4.3 Step D) against the complex128 oracle, and against
the table-driven sweep on the same plan.  Both paths run the same ops in the
same order with the same gate bodies; only the compiler's fused
multiply-adds may differ, so the two agree far inside the oracle tolerance."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2509_14098_amd as Q
import workloads as W
from spec_cases import RANDOM_CASES, SHAPES

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-5          # max-abs amplitude error against the oracle
SAME = 2e-6         # max-abs difference between the specialised and the table-driven sweep


@pytest.fixture(scope="module")
def sim():
    s = Q.Simulator(0)
    yield s
    s.close()


def both(sim, n, gates, k, tile=None, theta=None, flags=0, psi0=None):
    """Apply the plan table-driven, then specialised; returns both states."""
    plan = sim.partition(n, gates, k, flags, tile)
    try:
        out = []
        for spec in (False, True):
            if spec:
                secs = sim.specialise(plan)
                assert plan.info["specialised"] == 1 and secs > 0
            psi = sim.zero_state(n) if psi0 is None else psi0.clone()
            sim.apply(plan, psi, theta)
            torch.cuda.synchronize()
            out.append(psi.cpu().numpy())
        return out[0], out[1], plan.info
    finally:
        plan.close()


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128))))


@pytest.mark.parametrize("n,ng,k,tile", RANDOM_CASES)
def test_specialised_random_circuits(sim, n, ng, k, tile):
    """Every gate kind (fixed and parameterised) at random positions."""
    theta = np.random.default_rng(n).uniform(-3, 3, size=5)
    gates = W.random_circuit(n, ng, seed=5000 + n, n_params=5)
    ref = oracle.apply(n, gates, theta)
    a, b, info = both(sim, n, gates, k, tile, theta)
    assert info["n_partitions"] >= 1
    assert maxabs(b, ref) <= TOL
    assert maxabs(a, b) <= SAME


@pytest.mark.parametrize("R,LW", SHAPES)
def test_specialised_every_kernel_shape(sim, R, LW):
    """Full tiles of every kernel shape up to 13 tile qubits, several tiles and
    tile-index qubits, against the oracle and the table-driven sweep."""
    n = R + LW + 2
    theta = np.random.default_rng(R * 16 + LW).uniform(-3, 3, size=4)
    # one register qubit holds a gate's local qubits only when at most one must be
    # local: no SWAP or dense two-qubit gate there (the planner would widen R)
    kinds = [k for k in W.KIND if k not in ("SWAP", "MAT2")] if R == 1 else None
    gates = W.random_circuit(n, 150, seed=6000 + 16 * R + LW, n_params=4, kinds=kinds)
    ref = oracle.apply(n, gates, theta)
    a, b, info = both(sim, n, gates, min(n, R + LW - 1, 9), (R, LW), theta)
    assert (info["reg_qubits"], info["log_threads"], info["tile_qubits"]) == (R, LW, R + LW)
    assert maxabs(b, ref) <= TOL
    assert maxabs(a, b) <= SAME


def test_specialised_c2_full(sim):
    """28-qubit brickwork at k = 10 (the benchmark plan): specialised against
    the table-driven sweep on the whole state and against the oracle's stored
    amplitudes."""
    g = np.load(os.path.join(GOLDEN, "c2.npz"))
    gates = W.brickwork_c2()
    assert W.circuit_hash(gates, 28) == g["circuit_sha256"].item().decode()
    plan = sim.partition(28, gates, 10)
    try:
        ref = sim.zero_state(28)
        sim.apply(plan, ref)
        sim.specialise(plan)
        psi = sim.zero_state(28)
        sim.apply(plan, psi)
        torch.cuda.synchronize()
        assert float((psi - ref).abs().max()) <= SAME
        del ref
        got = psi[torch.as_tensor(g["idx"], device=psi.device)].cpu().numpy()
        assert np.max(np.abs(got - g["amp"])) <= TOL
        z0 = float(sim.expect(W.z_on(0), psi, 28)[0])
        assert abs(z0 - float(g["z0"])) < 1e-5
    finally:
        plan.close()
        torch.cuda.empty_cache()


def test_specialised_maximum_size_34_qubits(sim):
    """34 qubits (128 GiB, 2^21 workgroups per sweep) on specialised kernels
    with 13-qubit tiles: a U3 layer against its product-state closed form on
    sampled amplitudes, then a brickwork and its inverse back to it."""
    n = 34
    torch.cuda.empty_cache()

    def spec_apply(gates, psi):
        plan = sim.partition(n, gates, 10, 0, (4, 9))
        try:
            sim.specialise(plan)
            sim.apply(plan, psi)
            torch.cuda.synchronize()
        finally:
            plan.close()

    layer, ang = W.u3_layer(n, seed=11)
    psi = sim.zero_state(n)
    spec_apply(layer, psi)
    idx = np.random.default_rng(5).integers(0, 1 << n, size=1024)
    got = psi[torch.as_tensor(idx, device=psi.device)].cpu().numpy()
    ref = np.ones(len(idx), complex)
    for q in range(n):
        b = (idx >> q) & 1
        ref *= np.where(b == 0, np.cos(ang[q, 0] / 2), np.exp(1j * ang[q, 1]) * np.sin(ang[q, 0] / 2))
    assert np.max(np.abs(got - ref)) < 1e-7
    body = W.brickwork_c3(n=n, layers=3, seed=12)
    spec_apply(body, psi)
    spec_apply(W.inverse_circuit(body), psi)
    back = psi[torch.as_tensor(idx, device=psi.device)].cpu().numpy()
    assert np.max(np.abs(back - ref)) < 1e-6
    del psi
    torch.cuda.empty_cache()


def test_specialised_reads_theta_at_apply_time(sim):
    """Parameterised rotations keep their matrices in device memory: one
    specialised plan, two parameter vectors, both against the oracle."""
    n = 14
    gates, npar = W.ansatz(n, 4)
    plan = sim.partition(n, gates, 10, 0, (4, 8))
    try:
        sim.specialise(plan)
        for seed in (1, 2):
            theta = W.ansatz_params(npar, seed=seed)
            psi = sim.zero_state(n)
            sim.apply(plan, psi, theta)
            torch.cuda.synchronize()
            assert maxabs(psi.cpu().numpy(), oracle.apply(n, gates, theta)) <= TOL
    finally:
        plan.close()


def test_specialised_forward_feeds_the_adjoint(sim):
    """Checkpoints written by the specialised sweeps equal the table-driven
    ones; the specialised adjoint walk gives the table-driven gradient and
    matches the oracle's adjoint."""
    n, npar = 16, 6
    theta = np.random.default_rng(7).uniform(-3, 3, size=npar)
    gates = W.random_circuit(n, 200, seed=3107, n_params=npar)
    H = W.zz_chain_plus_x(n, 0.5)
    e_ref, g_ref = oracle.adjoint(n, gates, theta, H)
    plan = sim.partition(n, gates, 9, Q.PLAN_GRAD, (4, 8))
    try:
        res = []
        for spec in (False, True):
            if spec:
                sim.specialise(plan)
            psi = sim.zero_state(n)
            ckpt = sim.checkpoints(plan)
            sim.apply(plan, psi, theta, ckpt)
            e, g = sim.adjoint_grad(plan, H, theta, psi, ckpt)
            torch.cuda.synchronize()
            res.append((ckpt.cpu().numpy(), float(e[0]), g.cpu().numpy()))
    finally:
        plan.close()
    assert maxabs(res[0][0], res[1][0]) <= SAME
    assert abs(res[0][1] - res[1][1]) < 1e-6 and np.max(np.abs(res[0][2] - res[1][2])) < 1e-5
    e, g = res[1][1], res[1][2]
    assert abs(e - e_ref) < 1e-4
    assert np.max(np.abs(g - g_ref[:len(g)])) < 1e-4


def test_specialised_c4_gradient(sim):
    """20-qubit RY.RZ + CX-ladder ansatz, 10 layers, 400 parameters, through
    the autograd Function on a specialised plan (forward sweeps and adjoint
    walk generated): energy and every gradient entry against the oracle."""
    n = 20
    gates, npar = W.ansatz(n, 10)
    theta = W.ansatz_params(npar, seed=4)
    H = W.zz_chain_plus_x(n, 0.5)
    e_ref, g_ref = oracle.adjoint(n, gates, theta, H)
    plan = sim.partition(n, gates, 10, Q.PLAN_GRAD)
    try:
        sim.specialise(plan)
        th = torch.as_tensor(theta, device="cuda").clone().requires_grad_(True)
        e = Q.Energy.apply(th, sim, plan, H)
        e.backward()
        g = th.grad.cpu().numpy()
    finally:
        plan.close()
    assert abs(float(e.detach()) - e_ref) < 1e-4
    assert np.max(np.abs(g - g_ref)) < 1e-4


def test_specialised_distributed_plan(sim):
    """A plan with the distributed level (remap SWAP partitions included)."""
    n, gl = 16, 2
    gates = W.random_circuit(n, 250, seed=611)
    ref = oracle.apply(n, gates)
    plan = sim.partition_distributed(n, gates, gl, 8, 0, (4, 8))
    try:
        sim.specialise(plan)
        psi = sim.zero_state(n)
        sim.apply(plan, psi)
        torch.cuda.synchronize()
        assert maxabs(psi.cpu().numpy(), ref) <= TOL
    finally:
        plan.close()


def test_specialised_qft_and_empty_circuit(sim):
    """Diagonal-heavy partitions (QFT of a basis state against its closed
    form) and a circuit with no gates (the state is left as it is)."""
    n = 16
    N = 1 << n
    x = (5 * N) // 7
    psi0 = torch.zeros(N, dtype=torch.complex64, device="cuda")
    psi0[x] = 1
    a, b, _ = both(sim, n, W.qft(n), 10, (4, 8), psi0=psi0)
    ref = np.exp(2j * np.pi * x * np.arange(N) / N) / np.sqrt(N)
    assert maxabs(b, ref) <= TOL and maxabs(a, b) <= SAME
    rnd = torch.randn(1 << 10, dtype=torch.complex64, device="cuda")
    a, b, info = both(sim, 10, W.ghz(10)[:0], 6, psi0=rnd)
    assert np.array_equal(b, rnd.cpu().numpy()) and np.array_equal(a, b)


def test_specialised_kernels_from_the_code_object_cache(sim, tmp_path, monkeypatch):
    """A plan specialised with QSV_KERNEL_CACHE set leaves its code objects
    there; the same plan built again loads them (QSV_KERNEL_CACHE_ONLY: no
    compiler started) and reaches the oracle's state."""
    n = 15
    theta = np.random.default_rng(9).uniform(-3, 3, size=4)
    gates = W.random_circuit(n, 200, seed=9109, n_params=4)
    ref = oracle.apply(n, gates, theta)
    monkeypatch.setenv("QSV_KERNEL_CACHE", str(tmp_path))
    for cache_only in ("0", "1"):
        monkeypatch.setenv("QSV_KERNEL_CACHE_ONLY", cache_only)
        plan = sim.partition(n, gates, 9, 0, (4, 8))
        try:
            sim.specialise(plan)
            psi = sim.zero_state(n)
            sim.apply(plan, psi, theta)
            torch.cuda.synchronize()
            assert maxabs(psi.cpu().numpy(), ref) <= TOL
        finally:
            plan.close()
        assert any(p.suffix == ".co" for p in tmp_path.iterdir())


def test_autotuner_times_specialised_candidates(sim):
    """QSV_PLAN_TUNE_SPECIALISED with k given: only tile shapes of at most 13
    qubits at that k are timed, the plan takes the fastest, and its
    specialised sweeps match the oracle."""
    n = 18
    gates = W.random_circuit(n, 200, seed=8101, n_params=3)
    theta = np.random.default_rng(3).uniform(-3, 3, size=3)
    plan = sim.partition(n, gates, 8, Q.PLAN_TUNE_SPECIALISED)
    try:
        cand = Q.qsv_last_autotune()
        assert len(cand) >= 2 and all(c[0] == 8 and c[1] + c[2] <= 13 for c in cand)
        best = min(cand, key=lambda c: c[3])
        assert (plan.info["k_local"], plan.info["reg_qubits"], plan.info["log_threads"]) == tuple(best[:3])
        sim.specialise(plan)
        psi = sim.zero_state(n)
        sim.apply(plan, psi, theta)
        torch.cuda.synchronize()
        assert maxabs(psi.cpu().numpy(), oracle.apply(n, gates, theta)) <= TOL
    finally:
        plan.close()


def test_specialise_errors(sim):
    """Tiles above 64 KiB of LDS are not specialised; a host-only plan has
    nothing to load on a device.  Each error leaves the plan usable by the
    table-driven sweep."""
    big = sim.partition(16, W.random_circuit(16, 50, seed=3), 12, 0, (5, 9))
    try:
        with pytest.raises(Q.QsvError) as e:
            sim.specialise(big)
        assert e.value.code == -6 and big.info["specialised"] == 0
        psi = sim.zero_state(16)
        sim.apply(big, psi)
        torch.cuda.synchronize()
        assert maxabs(psi.cpu().numpy(), oracle.apply(16, W.random_circuit(16, 50, seed=3))) <= TOL
    finally:
        big.close()
    host = Q.qsv_partition(None, 8, W.ghz(8), None, 4, 0, None)
    try:
        with pytest.raises(Q.QsvError) as e:
            Q.qsv_plan_specialise(sim.ctx, host)
        assert e.value.code == -5
    finally:
        Q.qsv_plan_destroy(host)


def test_specialise_async_switches_during_applies(sim):
    """qsv_plan_specialise_async: applies run at once (table-driven while the
    compile is pending, specialised sweeps once it has finished, possibly
    within one apply); every state equals the oracle's, the plan ends up
    specialised, and qsv_plan_specialise then returns without compiling."""
    n = 24
    gates = W.brickwork_c3(n=n, layers=30, seed=21)
    ref = oracle.apply(n, gates)
    plan = sim.partition(n, gates, 10, 0, (4, 9))
    try:
        sim.specialise_async(plan)
        seen = set()
        for _ in range(400):  # bounded: the compile takes seconds, an apply milliseconds
            psi = sim.zero_state(n)
            sim.apply(plan, psi)
            torch.cuda.synchronize()
            assert maxabs(psi.cpu().numpy(), ref) <= TOL
            spec = plan.refresh()["specialised"]
            seen.add(spec)
            if spec:
                break
        if not plan.info["specialised"]:
            sim.specialise(plan)  # waits for the compile
        assert plan.refresh()["specialised"] == 1
        psi = sim.zero_state(n)
        sim.apply(plan, psi)
        torch.cuda.synchronize()
        assert maxabs(psi.cpu().numpy(), ref) <= TOL
        print(f"async specialise: table-driven applies seen {0 in seen}", flush=True)
    finally:
        plan.close()


def test_specialise_async_gradient_and_destroy_while_pending(sim):
    """A gradient plan specialised in the background gives the oracle's
    gradient before and after its kernels arrive; a plan destroyed while its
    compile runs waits for it."""
    n = 12
    gates, npar = W.ansatz(n, 4)
    theta = W.ansatz_params(npar, seed=8)
    H = W.zz_chain_plus_x(n, 0.5)
    e_ref, g_ref = oracle.adjoint(n, gates, theta, H)
    plan = sim.partition(n, gates, 8, Q.PLAN_GRAD, (3, 6))
    th = sim.theta(theta)
    try:
        sim.specialise_async(plan)
        for _ in range(2):
            psi = sim.zero_state(n)
            ckpt = sim.checkpoints(plan)
            sim.apply(plan, psi, th, ckpt)
            e, g = sim.adjoint_grad(plan, H, th, psi, ckpt)
            torch.cuda.synchronize()
            assert abs(float(e[0]) - e_ref) < 1e-5
            assert float(np.max(np.abs(g.cpu().numpy() - g_ref))) < 1e-4
            sim.specialise(plan)
            assert plan.refresh()["specialised"] == 1
    finally:
        plan.close()
    other = sim.partition(n, gates, 8, Q.PLAN_GRAD, (3, 6))
    sim.specialise_async(other)
    other.close()  # joins the pending compile


# ---------------------------------------------------------------- batched plans

def _batched_case(n, seed):
    """Circuits of several structures in one batch: ansatz instances of
    depths 1-3 (each depth twice, so instances share tables), an empty
    circuit, and random circuits over every gate kind with parameters."""
    rng = np.random.default_rng(seed)
    circs, thetas = [], []
    for d in (1, 2, 3, 2, 1, 3):
        g, npar = W.ansatz(n, d)
        circs.append(g)
        thetas.append(rng.uniform(-np.pi, np.pi, size=npar))
    a, _ = W.ansatz(n, 1)
    circs.append(a[:0])
    thetas.append(np.zeros(0))
    for i in range(3):
        circs.append(W.random_circuit(n, 60, seed=seed + i, n_params=3))
        thetas.append(rng.uniform(-3, 3, size=3))
    gates = np.concatenate(circs)
    off = np.concatenate([[0], np.cumsum([len(c) for c in circs])])
    return circs, thetas, gates, off, np.concatenate(thetas)


def test_specialised_batched_forward_and_gradient(sim):
    """qsv_plan_specialise on a batched plan: one persistent kernel with every
    circuit structure compiled in runs the forward launches.  Final states
    against the oracle and against the table-driven kernel; energies and
    gradients (adjoint walk from the specialised forward's states, in two
    launches, and from given states) against the oracle's adjoint."""
    n = 6
    circs, thetas, gates, off, theta = _batched_case(n, 70)
    B = len(circs)
    H = W.zz_chain_plus_x(n, 0.5)
    plan = sim.partition(n, gates, 0, Q.PLAN_GRAD, None, circ_offsets=off)
    try:
        ref_psi = torch.empty((B, 1 << n), dtype=torch.complex64, device="cuda")
        sim.apply(plan, ref_psi, theta)
        secs = sim.specialise(plan)
        assert plan.info["specialised"] == 1 and secs > 0
        psi = torch.empty((B, 1 << n), dtype=torch.complex64, device="cuda")
        sim.apply(plan, psi, theta)
        e1, g1 = sim.adjoint_grad(plan, H, theta)         # specialised forward, then the adjoint walk
        e2, g2 = sim.adjoint_grad(plan, H, theta, psi)    # from the given final states
        torch.cuda.synchronize()
    finally:
        plan.close()
    psi, ref_psi = psi.cpu().numpy(), ref_psi.cpu().numpy()
    assert maxabs(psi, ref_psi) <= SAME
    assert np.array_equal(e1.cpu().numpy(), e2.cpu().numpy())
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())
    e1, g1 = e1.cpu().numpy(), g1.cpu().numpy()
    p0 = 0
    for b in range(B):
        assert maxabs(psi[b], oracle.apply(n, circs[b], thetas[b])) <= TOL, b
        e_ref, g_ref = oracle.adjoint(n, circs[b], thetas[b], H)
        assert abs(e1[b] - e_ref) < 1e-5, b
        if len(thetas[b]):
            assert np.max(np.abs(g1[p0:p0 + len(thetas[b])] - g_ref)) < 1e-4, b
        p0 += len(thetas[b])


def test_specialised_batched_in_the_background(sim):
    """qsv_plan_specialise_async on a batched plan: forward launches run
    table-driven until the compile has finished, then on the specialised
    kernel; every launch's states equal the oracle's."""
    n = 8
    circs, thetas, gates, off, theta = _batched_case(n, 90)
    B = len(circs)
    plan = sim.partition(n, gates, 0, Q.PLAN_GRAD, None, circ_offsets=off)
    try:
        sim.specialise_async(plan)
        psi = torch.empty((B, 1 << n), dtype=torch.complex64, device="cuda")
        outs = []
        for _ in range(3):
            sim.apply(plan, psi, theta)
            outs.append(psi.cpu().numpy())
        sim.specialise(plan)  # waits for the compile
        assert plan.info["specialised"] == 1
        sim.apply(plan, psi, theta)
        outs.append(psi.cpu().numpy())
    finally:
        plan.close()
    for out in outs:
        for b in range(B):
            assert maxabs(out[b], oracle.apply(n, circs[b], thetas[b])) <= TOL, b
