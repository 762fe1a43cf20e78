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


# ---------------------------------------------------------------------------
# Hand-derived pins of the greedy's ranking (Section 4.2, Fig. 5 step 3: take
# the frontier gates of highest closeness centrality; ties by lower
# critical-path length, then lower gate index).  In each circuit two or more
# ready gates compete for the last free local qubit, so the rule fixes which
# gates share a partition.  Nodes: psi = 0, gate i = node i + 1; N = G + 1;
# CC = |RN|^2 / (N dist) with dist = sum over RN of (l_w - l_v).  The values
# below were worked out by hand (the derivations are listed with the
# partitioner's readings); the tests check the oracle against them.

def _mk(specs):
    return W.make_gates(specs)


# (name, n, k, gate specs, l per node, CC per node, expected partitions)
RANKING_CASES = [
    # CC decides: g0 = H0 (RN {g2, g3}, dist 1 + 2, CC 4/15) beats g1 = H2
    # (a sink, CC 0); the SWAP(0,1) then fills the local set {0, 1}, and H2
    # is left for a second partition.  Ascending CC would start with H2.
    ("cc", 3, 2, [("H", (0,)), ("H", (2,)), ("SWAP", (0, 1)), ("H", (1,))],
     [0, 1, 1, 2, 3],
     [Fraction(16, 35), Fraction(4, 15), Fraction(0), Fraction(1, 5), Fraction(0)],
     [([0, 1], [0, 2, 3]), ([0, 2], [1])]),
    # Critical-path length decides: after H0, the sinks SWAP(0,1) (l 2) and
    # H2 (l 1) tie at CC 0; the lower l takes qubit 2, so the SWAP waits.
    # Preferring the lower index (or the higher l) would take the SWAP.
    ("l", 3, 2, [("H", (0,)), ("SWAP", (0, 1)), ("H", (2,))],
     [0, 1, 2, 1],
     [Fraction(9, 16), Fraction(1, 4), Fraction(0), Fraction(0)],
     [([0, 2], [0, 2]), ([0, 1], [1])]),
    # Gate index decides: after H0 (CC 1/5), the sinks H1 and H2 tie at CC 0
    # and l 1; the lower index takes qubit 1, then the second H0 (l 2) fits.
    ("index", 3, 2, [("H", (0,)), ("H", (1,)), ("H", (2,)), ("H", (0,))],
     [0, 1, 1, 1, 2],
     [Fraction(16, 25), Fraction(1, 5), Fraction(0), Fraction(0), Fraction(0)],
     [([0, 1], [0, 1, 3]), ([0, 2], [2])]),
    # Centrality, not reach: a chain of five H on qubit 0 gives its head four
    # downstream gates at distances 1..4 (CC 16/90 = 8/45), SWAP(1,2) has two
    # at distance 1 (CC 4/18 = 2/9 > 8/45).  The SWAP opens the first
    # partition with its two followers; ranking by reach or ascending CC
    # would open with the chain instead.
    ("reach", 3, 2, [("H", (0,))] * 5 + [("SWAP", (1, 2)), ("H", (1,)), ("H", (2,))],
     [0, 1, 2, 3, 4, 5, 1, 2, 2],
     [Fraction(16, 45), Fraction(8, 45), Fraction(1, 6), Fraction(4, 27), Fraction(1, 9), Fraction(0),
      Fraction(2, 9), Fraction(0), Fraction(0)],
     [([1, 2], [5, 6, 7]), ([0, 1], [0, 1, 2, 3, 4])]),
]


@pytest.mark.parametrize("case", RANKING_CASES, ids=[c[0] for c in RANKING_CASES])
def test_ranking_pins_hand_derived(case):
    _, n, k, specs, l_ref, cc_ref, parts_ref = case
    gates = _mk(specs)
    assert C.critical_path_lengths(n, gates) == l_ref
    assert [c for _, _, c in C.closeness(n, gates)] == cc_ref
    parts = C.greedy_partition(n, gates, k)
    assert parts == parts_ref
    C.check_partition(n, gates, k, parts)
    # every candidate ordering still reaches the sequential state
    order = [g for _, p in parts for g in p]
    assert np.max(np.abs(oracle.apply(n, gates) - oracle.apply(n, gates[order]))) < 1e-13


def test_controls_join_the_local_set_only_when_there_is_room():
    """Section 4.2's second exemption: after H1 and H2 fill the local set
    {1, 2}, CX(0 -> 1) still joins the partition (only its target must be
    local) and its control stays global."""
    gates = _mk([("H", (1,)), ("CX", (0, 1)), ("H", (2,))])
    assert C.greedy_partition(3, gates, 2) == [([1, 2], [0, 2, 1])]
