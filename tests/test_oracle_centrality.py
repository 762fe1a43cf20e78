"""Pins of the graph side of the oracle: the paper's printed values (Section
4.1: l_H = 1, l_CX = 2 on the driving example; Section 4.3 / Fig. 6: the
two-level partition tree of GHZ-3 with L0 global in i_2 and R0 global in i_0),
the paper's own recursion for reachable sets and distances (Eq. 11-13 with
both double-count branches), NetworkX closeness centrality, the locality
exemptions (Section 4.2) and the invariants any valid partition satisfies."""
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import centrality as C


def test_worked_example_critical_path():
    l = C.critical_path_lengths(3, W.ghz(3))
    assert l[1] == 1 and l[2] == 2  # H, first CX
    preds, _ = C.contraction_graph(3, W.ghz(3))
    assert 0 in preds[2]  # direct edge between the first CX and psi


def test_worked_example_partition_tree():
    parts = C.greedy_partition(3, W.ghz(3), k=2)
    assert parts == [([0, 1], [0, 1]), ([1, 2], [2])]


def _paper_recursion(n, gates, threshold):
    """Eq. 11-13: walk nodes from the last to the first; start from one
    downstream neighbour v_j, add the others v_k, and correct double counts by
    subtracting overlapping distances (overlap below threshold) or by adding
    the symmetric difference and halving (overlap above threshold)."""
    _, succs = C.contraction_graph(n, gates)
    l = C.critical_path_lengths(n, gates)
    N = len(gates) + 1
    RN = [set() for _ in range(N)]
    dist = [0] * N
    for v in reversed(range(N)):
        kids = sorted(succs[v])
        if not kids:
            continue
        j = kids[0]
        RN[v] = {j} | RN[j]
        dist[v] = (1 + len(RN[j])) * abs(l[v] - l[j]) + dist[j]
        for k in kids[1:]:
            add = {k} | RN[k]
            d_add = (1 + len(RN[k])) * abs(l[v] - l[k]) + dist[k]
            overlap = RN[v] & add
            dsum = lambda s: sum(l[w] - l[v] for w in s)
            if len(overlap) < threshold:
                dist[v] = dist[v] + d_add - dsum(overlap)
            else:
                dist[v] = (dist[v] + d_add + dsum(RN[v] ^ add)) // 2
            RN[v] |= add
    return RN, dist


@pytest.mark.parametrize("seed", range(12))
def test_closeness_bruteforce_vs_paper_recursion(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    gates = W.random_circuit(n, int(rng.integers(1, 45)), seed=seed)
    ref = C.closeness(n, gates)
    for thr in (0, 10 ** 9):
        RN, dist = _paper_recursion(n, gates, thr)
        assert [(len(r), d) for r, d in zip(RN, dist)] == [(a, b) for a, b, _ in ref]


@pytest.mark.parametrize("seed", range(6))
def test_closeness_vs_networkx(seed):
    """CC_paper = networkx closeness on the reversed graph (outward distances,
    edge weight l_v - l_u, Wasserman-Faust on) times (N-1)/N."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    gates = W.random_circuit(n, int(rng.integers(2, 40)), seed=100 + seed)
    _, succs = C.contraction_graph(n, gates)
    l = C.critical_path_lengths(n, gates)
    G = nx.DiGraph()
    G.add_nodes_from(range(len(gates) + 1))
    for u, vs in enumerate(succs):
        for v in vs:
            G.add_edge(u, v, weight=l[v] - l[u])
    ccnx = nx.closeness_centrality(G.reverse(), distance="weight", wf_improved=True)
    N = len(gates) + 1
    for v, (_, _, cc) in enumerate(C.closeness(n, gates)):
        assert abs(float(cc) - ccnx[v] * (N - 1) / N) < 1e-12


def test_worked_example_centrality_values():
    cc = [c for _, _, c in C.closeness(3, W.ghz(3))]
    assert cc == [Fraction(3, 8), Fraction(1, 3), Fraction(1, 4), Fraction(0)]


def test_locality_exemptions():
    mk = W.make_gates
    # a phase gate has only diagonal entries (Section 4.2 first exemption)
    assert C.required_local(mk([("P", (3,), (0.4,))])[0]) == ()
    assert C.required_local(mk([("RZ", (3,), (0.4,))])[0]) == ()
    assert C.required_local(mk([("CZ", (1, 4))])[0]) == ()
    assert C.required_local(mk([("RZZ", (1, 4), (0.3,))])[0]) == ()
    # controlled gates: only the target must be local (second exemption)
    assert C.required_local(mk([("CX", (5, 2))])[0]) == (2,)
    assert C.required_local(mk([("CY", (0, 2))])[0]) == (2,)
    # everything else needs all its qubits
    assert C.required_local(mk([("H", (3,))])[0]) == (3,)
    assert C.required_local(mk([("SWAP", (1, 4))])[0]) == (1, 4)
    # a parameterised RX is dense for a generic angle even if the current angle is 0
    assert C.required_local(mk([("RX", (2,), (), 0)])[0], np.zeros(1)) == (2,)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("k", [2, 3, 5])
def test_partition_invariants_and_sequential_result(seed, k):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(2, 9))
    theta = rng.uniform(-3, 3, size=3)
    gates = W.random_circuit(n, int(rng.integers(1, 70)), seed=200 + seed, n_params=3)
    parts = C.greedy_partition(n, gates, k, theta)
    C.check_partition(n, gates, k, parts, theta)
    order = [g for _, p in parts for g in p]
    a = oracle.apply(n, gates, theta)
    b = oracle.apply(n, gates[order], theta)
    assert np.max(np.abs(a - b)) < 1e-13  # partitioned order reaches the sequential result


def test_partition_of_benchmark_circuit_c1():
    g = W.brickwork_c1()
    parts = C.greedy_partition(12, g, 8)
    C.check_partition(12, g, 8, parts)
    assert len(parts) >= 2
