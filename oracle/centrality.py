"""ORACLE — test infrastructure only (see ``oracle/__init__.py``).

Brute-force versions of the paper's graph analysis, written for clarity:

* the contraction graph (Section 3.2, Section 4.1, Fig. 4): node 0 is the
  state tensor psi, node i+1 is gate i; for every qubit of a gate there is an
  edge from the previous tensor on that qubit (psi if none) to the gate;
* the critical-path length l of each node (Section 4.1: l(psi) = 0 and a gate
  sits one step after the latest tensor it shares a dimension with);
* reachable nodes RN(v) (every node downstream of v), dist(v) as the sum of
  path lengths to them, measured in critical-path levels (Eq. 12-13: a path
  v -> w has length l_w - l_v), and closeness centrality Eq. 10 with the
  Wasserman-Faust factor |RN|/N, i.e. CC = |RN|^2 / (N dist), taken as 0 when
  RN is empty;
* the greedy frontier partition (Section 4.2, Fig. 5 step 3, and the two
  locality exemptions for diagonal gates and non-local controls).

All quantities are integers or exact fractions.

Pins: the worked example (GHZ-3: critical-path lengths, CC values and the
partition tree of Fig. 5), CC against networkx's closeness centrality and
against the paper's recursive form of RN and dist, and four small circuits
worked out by hand in which competing frontier gates are ordered by CC, then
by critical-path length, then by index (each rule, reversed, changes one of
their partitions).  On large circuits the tests check the invariants every
valid partition meets (locality, dependency order, the sequential state).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import gate_matrix

_ONE_QUBIT_KINDS = set(range(1, 15)) | {30}


def gate_qubits(g):
    if int(g["kind"]) in _ONE_QUBIT_KINDS:
        return (int(g["q0"]),)
    return (int(g["q0"]), int(g["q1"]))


def contraction_graph(n: int, gates):
    """Predecessor and successor sets, node 0 = psi, node i+1 = gate i."""
    N = len(gates) + 1
    preds = [set() for _ in range(N)]
    succs = [set() for _ in range(N)]
    last = [0] * n  # latest tensor touching each qubit
    for i, g in enumerate(gates):
        v = i + 1
        for q in gate_qubits(g):
            u = last[q]
            preds[v].add(u)
            succs[u].add(v)
            last[q] = v
    return preds, succs


def critical_path_lengths(n: int, gates):
    preds, _ = contraction_graph(n, gates)
    l = [0] * (len(gates) + 1)
    for v in range(1, len(gates) + 1):
        l[v] = 1 + max(l[u] for u in preds[v])
    return l


def reachable(succs, v):
    """Every node downstream of v, by depth-first search."""
    seen, stack = set(), list(succs[v])
    while stack:
        w = stack.pop()
        if w not in seen:
            seen.add(w)
            stack.extend(succs[w])
    return seen


def closeness(n: int, gates):
    """Per node: (|RN|, dist, CC as a Fraction) with CC = |RN|^2 / (N dist)."""
    _, succs = contraction_graph(n, gates)
    l = critical_path_lengths(n, gates)
    N = len(gates) + 1
    out = []
    for v in range(N):
        rn = reachable(succs, v)
        dist = sum(l[w] - l[v] for w in rn)
        cc = Fraction(0) if not rn else Fraction(len(rn) ** 2, N * dist)
        out.append((len(rn), dist, cc))
    return out


def required_local(g, theta=None):
    """Qubits that must be local for the gate (Section 4.2 exemptions):
    a gate whose matrix has only diagonal non-zeros needs none; a gate that is
    the identity while one qubit is 0 and never changes that qubit (a control)
    needs only its other qubit; anything else needs all its qubits.
    Parameterised rotations are classified by the structure they have for a
    generic angle (RZ, RZZ diagonal; RX, RY dense)."""
    qs = gate_qubits(g)
    kind = int(g["kind"])
    if int(g["param"]) >= 0:
        return () if kind in (12, 25) else qs
    m = gate_matrix(g, theta)
    off = m - np.diag(np.diag(m))
    if not np.any(off != 0):
        return ()
    if len(qs) == 1:
        return qs
    # local index j = b(q0) + 2 b(q1)
    for c, (zero_ix, one_ix) in ((0, ((0, 2), (1, 3))), (1, ((0, 1), (2, 3)))):
        z, o = list(zero_ix), list(one_ix)
        blk_zero = m[np.ix_(z, z)]
        mixing = np.any(m[np.ix_(z, o)] != 0) or np.any(m[np.ix_(o, z)] != 0)
        if not mixing and np.all(blk_zero == np.eye(2)):
            return (qs[1 - c],)
    return qs


def greedy_partition(n: int, gates, k: int, theta=None):
    """Cut the circuit into partitions of at most k local qubits.

    From the moving frontier (the gates whose predecessors are all placed),
    repeatedly take the frontier gate of highest closeness centrality whose
    required-local qubits still fit into the current local set (ties: lower
    critical-path length, then lower index); the local set grows by the gate's
    qubits when they fit, otherwise by its required qubits only.  When no
    frontier gate fits, the partition is closed, its local set padded to
    min(k, n) qubits with the lowest-numbered free qubits, and a new one begins.
    Returns a list of (sorted local qubits, [gate indices in order]).
    """
    G = len(gates)
    if G == 0:
        return []
    k = min(k, n)
    cc = closeness(n, gates)
    l = critical_path_lengths(n, gates)
    preds, succs = contraction_graph(n, gates)
    req = [set(required_local(g, theta)) for g in gates]
    qub = [set(gate_qubits(g)) for g in gates]
    missing = [len(preds[v] - {0}) for v in range(G + 1)]  # unplaced predecessors
    ready = {v for v in range(1, G + 1) if missing[v] == 0}
    parts = []
    placed = 0
    while placed < G:
        S, part = set(), []
        while True:
            fits = [v for v in sorted(ready) if len(S | req[v - 1]) <= k]
            if not fits:
                break
            best = fits[0]
            for v in fits[1:]:
                a, b = (cc[v][2], -l[v], -v), (cc[best][2], -l[best], -best)
                if a > b:
                    best = v
            g = best - 1
            S = S | qub[g] if len(S | qub[g]) <= k else S | req[g]
            part.append(g)
            ready.discard(best)
            for w in succs[best]:
                missing[w] -= 1
                if missing[w] == 0:
                    ready.add(w)
            placed += 1
        for q in range(n):
            if len(S) >= k:
                break
            S.add(q)
        parts.append((sorted(S), part))
    return parts


def check_partition(n: int, gates, k: int, parts, theta=None):
    """Invariants of a valid partition (raises AssertionError):
    every gate exactly once, partition order is a topological order of the
    contraction graph, |S| = min(k, n), every gate's required qubits lie in S."""
    order = [g for _, p in parts for g in p]
    assert sorted(order) == list(range(len(gates))), "every gate exactly once"
    pos = {g: i for i, g in enumerate(order)}
    preds, _ = contraction_graph(n, gates)
    for g in range(len(gates)):
        for u in preds[g + 1]:
            if u > 0:
                assert pos[u - 1] < pos[g], "dependency order"
    for S, p in parts:
        assert len(S) == min(k, n) and len(set(S)) == len(S)
        for g in p:
            assert set(required_local(gates[g], theta)) <= set(S), "required qubits local"
    return True
