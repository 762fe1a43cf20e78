"""Host-side checks of the native library (no GPU needed): it loads, exports
every entry point the header declares, its partitioner (integer work) matches
the oracle's greedy partition exactly, its register stages satisfy the
partition invariants, and invalid input is rejected before any device work."""
import os
import re

import numpy as np
import pytest

import paper_2509_14098_amd as Q
import workloads as W
from oracle import centrality as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = Q.load_library()
    header = open(os.path.join(ROOT, "include", "qsv.h")).read()
    names = set(re.findall(r"^\s*(?:qsv_status|int32_t|const char \*)\s*(qsv_\w+)\s*\(", header, re.M))
    assert {"qsv_create", "qsv_partition", "qsv_apply", "qsv_expect", "qsv_adjoint_grad"} <= names
    for name in names:
        assert hasattr(lib, name), name
    assert set(Q.binding.EXPORTS) == names


def _plan_parts(plan, level=0):
    info = Q.qsv_plan_info(plan)
    count = info["n_partitions"] if level == 0 else info["n_stages"]
    return [Q.qsv_plan_partition(plan, 0, level, p) for p in range(count)]


def _compare(n, gates, k, theta=None, tile=None):
    plan = Q.qsv_partition(None, n, gates, None, k, 0, tile)
    try:
        mine = [(S, g) for S, g in _plan_parts(plan)]
        ref = C.greedy_partition(n, gates, k, theta)
        assert mine == [(list(S), list(g)) for S, g in ref]
        return plan
    except Exception:
        Q.qsv_plan_destroy(plan)
        raise


def test_worked_example_ghz3():
    plan = _compare(3, W.ghz(3), 2)
    Q.qsv_plan_destroy(plan)


@pytest.mark.parametrize("name,n,k", [("c1", 12, 6), ("c1", 12, 8), ("c2", 28, 10), ("c3", 32, 8), ("c3", 32, 10),
                                      ("c3", 32, 12), ("c4", 20, 10), ("qft", 28, 10), ("qft", 20, 6)])
def test_partition_matches_oracle_on_workloads(name, n, k):
    gates = {"c1": W.brickwork_c1, "c2": W.brickwork_c2, "c3": W.brickwork_c3,
             "c4": lambda: W.ansatz(20, 10)[0], "qft": lambda: W.qft(n)}[name]()
    tile = (5, 8) if k < 13 else (5, 9)
    plan = _compare(n, gates, k, tile=tile)
    info = Q.qsv_plan_info(plan)
    assert info["n_gates"] == len(gates)
    Q.qsv_plan_destroy(plan)


@pytest.mark.parametrize("seed", range(12))
def test_partition_matches_oracle_random(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 16))
    k = int(rng.integers(2, n + 1))
    if n > 12:  # a partition must leave room for at least one fill qubit in the default 12-qubit tile
        k = min(k, 11)
    theta = rng.uniform(-3, 3, size=4)
    gates = W.random_circuit(n, int(rng.integers(1, 150)), seed=500 + seed, n_params=4)
    plan = _compare(n, gates, k, theta)
    Q.qsv_plan_destroy(plan)


@pytest.mark.parametrize("seed", range(8))
def test_register_stages_are_valid_partitions(seed):
    """Level 2 (registers): every gate of a partition exactly once, in an
    order that respects the contraction graph, with its required qubits among
    the R register qubits of the stage."""
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(6, 22))
    gates = W.random_circuit(n, 200, seed=900 + seed, n_params=3)
    theta = rng.uniform(-3, 3, size=3)
    plan = Q.qsv_partition(None, n, gates, None, min(n, 9), 0, (4, 8))
    info = Q.qsv_plan_info(plan)
    parts = _plan_parts(plan, 0)
    stages = _plan_parts(plan, 1)
    R = info["reg_qubits"]
    order = [g for _, st in stages for g in st]
    # the stages of partition p cover exactly p's gates, before those of p+1
    pos = 0
    for _, p in parts:
        assert sorted(order[pos:pos + len(p)]) == sorted(p)
        pos += len(p)
    assert pos == len(order)
    C.check_partition(n, gates, n, [(list(range(n)), order)], theta)
    for S, st in stages:
        assert len(S) == R
        for g in st:
            assert set(C.required_local(gates[g], theta)) <= set(S)
    Q.qsv_plan_destroy(plan)


def test_gate_by_gate_plan():
    gates = W.brickwork_c1()
    plan = Q.qsv_partition(None, 12, gates, None, 8, Q.PLAN_GATE_BY_GATE)
    parts = _plan_parts(plan)
    assert [g for _, g in parts] == [[i] for i in range(len(gates))]
    assert all(len(S) == 8 for S, _ in parts)
    Q.qsv_plan_destroy(plan)


def test_plan_params_offsets():
    a, na = W.ansatz(5, 2)
    b, nb = W.ansatz(5, 3)
    gates = np.concatenate([a, b])
    plan = Q.qsv_partition(None, 5, gates, [0, len(a), len(a) + len(b)], 0, 0)
    assert Q.qsv_plan_params(plan, 0) == (0, na)
    assert Q.qsv_plan_params(plan, 1) == (na, nb)
    assert Q.qsv_plan_info(plan)["n_params"] == na + nb
    Q.qsv_plan_destroy(plan)


@pytest.mark.parametrize("case,code", [
    ("bad_qubit", -1), ("same_qubit", -1), ("param_on_h", -2), ("n0", -1), ("kneg", -1), ("kind", -1),
    ("batched_big", -1), ("k_too_big", -1), ("bad_offsets", -1),
])
def test_invalid_input_rejected(case, code):
    g = W.ghz(4)
    n, k, off = 4, 2, None
    if case == "bad_qubit":
        g["q1"][1] = 7
    elif case == "same_qubit":
        g["q1"][1] = g["q0"][1]
    elif case == "param_on_h":
        g["param"][0] = 0
    elif case == "n0":
        n = 0
    elif case == "kneg":
        k = -1
    elif case == "kind":
        g["kind"][2] = 99
    elif case == "batched_big":
        g = np.concatenate([W.ghz(15), W.ghz(15)])
        n, off = 15, [0, 15, 30]
    elif case == "k_too_big":
        g, n, k = W.ghz(20), 20, 13
    elif case == "bad_offsets":
        off = [0, 3, 2]
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_partition(None, n, g, off, k, 0, (5, 8))
    assert e.value.code == code


@pytest.mark.parametrize("name,n,layers,k", [("c2", 28, 120, 10), ("c3", 34, 100, 12)])
def test_partition_matches_oracle_above_5000_gates(name, n, layers, k):
    """Paper-scale gate counts: the 28-qubit brickwork generator at 120
    layers (5 055 gates) and the random-matching generator at 34 qubits and
    100 layers (5 100 gates), exact partitions against the oracle's greedy."""
    gen = W.brickwork_c2 if name == "c2" else W.brickwork_c3
    gates = gen(n=n, layers=layers, seed=11)
    assert len(gates) > 5000
    plan = _compare(n, gates, k, tile=(5, 8))
    Q.qsv_plan_destroy(plan)


def test_host_only_plans_reach_40_qubits():
    """Host-only plans (no device tables) take up to 40 qubits, device plans
    up to 35 (a 256 GiB complex64 state): the 40-qubit circuit whose 32-qubit
    rank share is the 60-layer random-matching workload plans on the host."""
    gates = W.brickwork_c3(n=40, layers=4, seed=3)
    plan = Q.qsv_partition(None, 40, gates, None, 10, 0, None)
    assert Q.qsv_plan_info(plan)["n_qubits"] == 40
    Q.qsv_plan_destroy(plan)
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_partition(None, 41, W.ghz(41), None, 10, 0, None)
    assert e.value.code == -1 and "40" in str(e.value)
    with pytest.raises(Q.QsvError):
        Q.qsv_partition_distributed(None, 41, W.ghz(41), 8)


@pytest.mark.parametrize("name,n,g", [("c2", 28, 4), ("c3", 32, 8), ("qft", 24, 4), ("rand", 18, 3),
                                      ("c3-40", 40, 8)])
def test_distributed_level_matches_oracle(name, n, g):
    """The distributed level is the same greedy with n - g local qubits (exact
    gate lists against the oracle's); every distributed partition's local set
    holds n - g qubits including its gates' required ones; the tile-level
    partitions under it keep every gate in order, with tiles inside one rank
    (low positions) except for the remap SWAPs."""
    gates = {"c2": W.brickwork_c2, "c3": W.brickwork_c3, "qft": lambda: W.qft(n),
             "rand": lambda: W.random_circuit(n, 300, seed=123),
             # the whole 40-qubit run: 256 ranks of 32 qubits
             "c3-40": lambda: W.brickwork_c3(n=40)}[name]()
    plan = Q.qsv_partition_distributed(None, n, gates, g)
    try:
        info = Q.qsv_plan_distributed_info(plan)
        assert info["n_global"] == g
        dist = [Q.qsv_plan_partition(plan, 0, -1, p) for p in range(info["n_dist_partitions"])]
        ref = C.greedy_partition(n, gates, n - g)
        assert [gl for _, gl in dist] == [list(p) for _, p in ref]
        prev, moved = set(range(n - g)), 0
        for S, gl in dist:
            assert len(S) == n - g
            for gi in gl:
                assert set(C.required_local(gates[gi])) <= set(S)
            moved += len(set(S) - prev)
            prev = set(S)
        assert moved <= info["exchange_swaps"] <= info["remap_swaps"]
        order = []
        for S, gl in _plan_parts(plan):
            logical = [x for x in gl if x >= 0]
            if logical:  # a compute partition: its tile stays inside a rank
                assert len(logical) == len(gl) and max(S) < n - g
            order += logical
        assert sorted(order) == list(range(len(gates)))  # every gate once (the greedy orders them)
        # and each distributed partition's gates run before the next one's
        where = {gi: i for i, (_, gl) in enumerate(dist) for gi in gl}
        assert [where[x] for x in order] == sorted(where[x] for x in order)
    finally:
        Q.qsv_plan_destroy(plan)


def test_distributed_rejects_too_many_global_qubits():
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_partition_distributed(None, 14, W.ghz(14), 3)  # 11 local qubits < default 12-qubit tile
    assert e.value.code == -1


def test_distributed_edge_cases():
    empty = Q.qsv_partition_distributed(None, 16, W.ghz(16)[:0], 2)
    try:
        assert Q.qsv_plan_distributed_info(empty) == dict(n_global=2, n_dist_partitions=1, exchange_swaps=0,
                                                          remap_swaps=0)
        assert Q.qsv_plan_info(empty)["n_partitions"] == 1  # one empty sweep
    finally:
        Q.qsv_plan_destroy(empty)
    gbg = Q.qsv_partition_distributed(None, 16, W.ghz(16), 2, 0, Q.PLAN_GATE_BY_GATE)
    try:
        info = Q.qsv_plan_distributed_info(gbg)
        assert Q.qsv_plan_info(gbg)["n_partitions"] == 16 + info["remap_swaps"]  # one sweep per gate or SWAP
    finally:
        Q.qsv_plan_destroy(gbg)
    for n, g in ((16, 0), (16, 5), (2, 1)):
        with pytest.raises(Q.QsvError):
            Q.qsv_partition_distributed(None, n, W.ghz(n), g)


# ---------------------------------------------------------------- specialised sweeps (compile only: no GPU here)

def test_specialise_compiles_without_a_gpu():
    """Generated kernels for every partition compile for gfx950 (hipRTC in the
    qsv_rtc helper); without a context nothing is loaded."""
    plan = Q.qsv_partition(None, 10, W.random_circuit(10, 120, seed=91, n_params=3), None, 6, 0, None)
    try:
        assert Q.qsv_plan_specialise(None, plan) > 0
        assert Q.qsv_plan_info(plan)["specialised"] == 0
    finally:
        Q.qsv_plan_destroy(plan)


def test_specialise_batched_compiles_without_a_gpu():
    """A batched plan's specialised program (one persistent kernel, every
    circuit structure compiled in) compiles for gfx950."""
    gates, _ = W.ansatz(6, 2)
    other, _ = W.ansatz(6, 1)
    plan = Q.qsv_partition(None, 6, np.concatenate([gates, other, gates]),
                           [0, len(gates), len(gates) + len(other), 2 * len(gates) + len(other)], 0, Q.PLAN_GRAD, None)
    try:
        assert Q.qsv_plan_specialise(None, plan) > 0
        assert Q.qsv_plan_info(plan)["specialised"] == 0
    finally:
        Q.qsv_plan_destroy(plan)


def test_specialise_rejections():
    big = Q.qsv_partition(None, 16, W.ghz(16), None, 12, 0, (5, 9))  # 14-qubit tiles: 128 KiB of LDS
    try:
        with pytest.raises(Q.QsvError) as e:
            Q.qsv_plan_specialise(None, big)
        assert e.value.code == -6
        with pytest.raises(Q.QsvError) as e:
            Q.qsv_plan_specialise(None, None)
        assert e.value.code == -1
    finally:
        Q.qsv_plan_destroy(big)


def test_compiler_helper_reports_errors(tmp_path):
    import subprocess
    helper = os.path.join(os.path.dirname(Q.library_path()), "qsv_rtc")
    bad = tmp_path / "bad.hip"
    bad.write_text('#include "spec.cuh"\nnot a declaration;\n')
    r = subprocess.run([helper, str(bad), str(tmp_path / "bad.co"), str(tmp_path / "bad.log")])
    assert r.returncode == 1
    assert "error" in (tmp_path / "bad.log").read_text()
    assert not (tmp_path / "bad.co").exists()
    r = subprocess.run([helper, str(bad)])
    assert r.returncode == 2


def test_specialise_survives_signals_during_compile():
    """A signal delivered to the host process while it waits for the compiler
    helpers (here an interval timer every 5 ms) neither fails the compile nor
    leaves a helper unreaped."""
    import signal
    hits = []
    old = signal.signal(signal.SIGALRM, lambda *_: hits.append(1))
    plan = Q.qsv_partition(None, 10, W.random_circuit(10, 150, seed=94, n_params=3), None, 6, 0, None)
    try:
        signal.setitimer(signal.ITIMER_REAL, 0.005, 0.005)
        try:
            assert Q.qsv_plan_specialise(None, plan) > 0
        finally:
            signal.setitimer(signal.ITIMER_REAL, 0)
    finally:
        signal.signal(signal.SIGALRM, old)
        Q.qsv_plan_destroy(plan)
    assert hits
    with pytest.raises(ChildProcessError):
        os.waitpid(-1, os.WNOHANG)  # no child left behind


def test_specialise_code_object_cache(tmp_path, monkeypatch):
    """QSV_KERNEL_CACHE keeps one code object per generated program; with
    QSV_KERNEL_CACHE_ONLY a plan whose programs are all cached specialises
    without starting a compiler, and any other plan is refused."""
    gates = W.random_circuit(9, 80, seed=92, n_params=2)
    monkeypatch.setenv("QSV_KERNEL_CACHE", str(tmp_path))
    plan = Q.qsv_partition(None, 9, gates, None, 6, 0, None)
    try:
        Q.qsv_plan_specialise(None, plan)
        files = sorted(p.name for p in tmp_path.iterdir())
        assert files and all(f.endswith(".co") and len(f) == 19 for f in files)
        monkeypatch.setenv("QSV_KERNEL_CACHE_ONLY", "1")
        Q.qsv_plan_specialise(None, plan)  # every program found: nothing compiled
        assert sorted(p.name for p in tmp_path.iterdir()) == files
    finally:
        Q.qsv_plan_destroy(plan)
    other = Q.qsv_partition(None, 9, W.random_circuit(9, 80, seed=93), None, 6, 0, None)
    try:
        with pytest.raises(Q.QsvError) as e:
            Q.qsv_plan_specialise(None, other)
        assert e.value.code == -4 and "not in the cache" in str(e.value)
    finally:
        Q.qsv_plan_destroy(other)


def test_tune_specialised_flag_on_host_only_plans():
    """QSV_PLAN_TUNE_SPECIALISED is a valid flag; without a context nothing is
    timed and the given k and the default tile shape are kept."""
    plan = Q.qsv_partition(None, 16, W.brickwork_c3(n=16, layers=4), None, 8, Q.PLAN_TUNE_SPECIALISED, None)
    try:
        info = Q.qsv_plan_info(plan)
        assert (info["k_local"], info["reg_qubits"], info["log_threads"]) == (8, 4, 8)
    finally:
        Q.qsv_plan_destroy(plan)
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_partition(None, 16, W.ghz(16), None, 8, 8, None)  # no such flag
    assert e.value.code == -1


def test_planner_ranking_on_hand_derived_cases():
    """The native planner reaches the hand-derived partitions in which
    closeness centrality, then critical-path length, then gate index decide
    between competing frontier gates (the same cases pin the oracle)."""
    from test_oracle_centrality import RANKING_CASES
    for name, n, k, specs, _, _, parts_ref in RANKING_CASES:
        plan = Q.qsv_partition(None, n, W.make_gates(specs), None, k, 0, (1, 6))
        try:
            assert [(list(S), list(g)) for S, g in _plan_parts(plan)] == parts_ref, name
        finally:
            Q.qsv_plan_destroy(plan)
