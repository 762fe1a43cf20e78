"""Circuit and observable descriptions plus the seeded generators of the
benchmark workloads.

A circuit is a flat, ordered list of gates on given qubits (the paper's
Section 4.1 view of an OpenQASM program).  It is stored as a numpy structured
array whose layout is the ``qsv_gate`` record of the C interface::

    int32 kind; int32 q0; int32 q1; int32 param; double angle[3]; double mat[32];

* one-qubit gates: ``q0`` is the target, ``q1 = -1``;
* controlled gates (CX, CY, CZ, CP): ``q0`` is the control, ``q1`` the target;
* SWAP, RZZ: the two qubits, order irrelevant;
* MAT2: a 4x4 matrix on local index ``j = b(q0) + 2*b(q1)``;
* ``param >= 0`` (RX, RY, RZ, RZZ only) takes the angle from ``theta[param]``;
  otherwise the angle is ``angle[0]`` (U3 uses ``angle[0..2] = theta, phi, lambda``);
* MAT1/MAT2 carry a row-major complex matrix as (re, im) pairs in ``mat``.

Qubit ``q`` is bit ``q`` of the amplitude index (the column-major stacking of
the paper's Eq. 4 / Eq. 7).

An observable is a real-weighted sum of Pauli strings, each stored as
``(coeff, x_mask, z_mask)``: bit q of ``x_mask`` is set for X or Y on qubit q,
bit q of ``z_mask`` for Z or Y.

Nothing here evaluates gates: the generators only draw angles and qubits.
"""
from __future__ import annotations

import hashlib

import numpy as np

GATE_DTYPE = np.dtype([
    ("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("param", "<i4"),
    ("angle", "<f8", (3,)), ("mat", "<f8", (32,)),
], align=True)
assert GATE_DTYPE.itemsize == 296

PAULI_DTYPE = np.dtype([("coeff", "<f8"), ("x_mask", "<u8"), ("z_mask", "<u8")], align=True)

KIND = dict(H=1, X=2, Y=3, Z=4, S=5, SDG=6, T=7, TDG=8, SX=9,
            RX=10, RY=11, RZ=12, P=13, U3=14,
            CX=20, CY=21, CZ=22, CP=23, SWAP=24, RZZ=25,
            MAT1=30, MAT2=31)
KIND_NAME = {v: k for k, v in KIND.items()}
ONE_QUBIT = {"H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY", "RZ", "P", "U3", "MAT1"}
PARAM_KINDS = {"RX", "RY", "RZ", "RZZ"}


def make_gates(specs) -> np.ndarray:
    """Build a gate array from tuples ``(name, qubits, angles=(), param=-1, mat=None)``."""
    out = np.zeros(len(specs), dtype=GATE_DTYPE)
    for i, sp in enumerate(specs):
        name, qubits = sp[0], sp[1]
        angles = sp[2] if len(sp) > 2 else ()
        param = sp[3] if len(sp) > 3 else -1
        mat = sp[4] if len(sp) > 4 else None
        out[i]["kind"] = KIND[name]
        out[i]["q0"] = qubits[0]
        out[i]["q1"] = qubits[1] if len(qubits) > 1 else -1
        out[i]["param"] = param
        a = np.zeros(3)
        a[:len(angles)] = angles
        out[i]["angle"] = a
        if mat is not None:
            m = np.asarray(mat, dtype=np.complex128).reshape(-1)
            buf = np.zeros(32)
            buf[0:2 * m.size:2] = m.real
            buf[1:2 * m.size:2] = m.imag
            out[i]["mat"] = buf
    return out


def circuit_hash(gates: np.ndarray, n_qubits: int, extra: bytes = b"") -> str:
    h = hashlib.sha256()
    h.update(np.int64(n_qubits).tobytes())
    h.update(np.ascontiguousarray(gates).tobytes())
    h.update(extra)
    return h.hexdigest()


# ---------------------------------------------------------------- small circuits

def ghz(n: int) -> np.ndarray:
    """The paper's driving example (Section 4.1 listing) extended to n qubits:
    H on qubit 0, then a CX chain."""
    return make_gates([("H", (0,))] + [("CX", (q, q + 1)) for q in range(n - 1)])


def uniform_h(n: int) -> np.ndarray:
    return make_gates([("H", (q,)) for q in range(n)])


def u3_layer(n: int, seed: int):
    """One U3 per qubit with angles iid U[0, 2pi); returns (gates, angles[n,3])."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2 * np.pi, size=(n, 3))
    return make_gates([("U3", (q,), tuple(ang[q])) for q in range(n)]), ang


def qft(n: int) -> np.ndarray:
    """Quantum Fourier transform from its textbook circuit, for the bit order
    used here (qubit q is bit q of the index): qubits from the highest down,
    each gets H and then controlled phases 2 pi / 2^(d+1) from every lower
    qubit at distance d; finally the qubit order is reversed with SWAPs.  It
    maps |x> to 2^(-n/2) sum_y exp(2 pi i x y / 2^n) |y>.  A diagonal-heavy
    workload: n(n-1)/2 of its gates are controlled phases, which the
    partitioner does not count against k."""
    specs = []
    for j in range(n - 1, -1, -1):
        specs.append(("H", (j,)))
        for m in range(j - 1, -1, -1):
            specs.append(("CP", (m, j), (np.pi / 2 ** (j - m),)))
    for i in range(n // 2):
        specs.append(("SWAP", (i, n - 1 - i)))
    return make_gates(specs)


# ---------------------------------------------------------------- benchmark workloads

def brickwork_c1(n: int = 12, layers: int = 20, seed: int = 1) -> np.ndarray:
    """U3(theta, phi, lambda) on every qubit, angles iid U[0, 2pi) drawn in
    (layer, qubit, theta/phi/lambda) order, then CZ on pairs (a, a+1) with
    a = layer mod 2, layer mod 2 + 2, ..."""
    rng = np.random.default_rng(seed)
    specs = []
    for layer in range(layers):
        ang = rng.uniform(0.0, 2 * np.pi, size=(n, 3))
        specs += [("U3", (q,), tuple(ang[q])) for q in range(n)]
        specs += [("CZ", (a, a + 1)) for a in range(layer % 2, n - 1, 2)]
    return make_gates(specs)


def brickwork_c2(n: int = 28, layers: int = 40, seed: int = 2, p_long: float = 0.05) -> np.ndarray:
    """U3 on all qubits, then nearest-neighbour pairs (a, a+1), a = layer mod 2
    + 2j: CZ on even layers, CX(a -> a+1) on odd layers.  After each
    nearest-neighbour gate, with probability ``p_long`` a CX(c, t) with
    (c, t) uniform over ordered pairs with |c - t| >= 2 is appended."""
    rng = np.random.default_rng(seed)
    long_pairs = [(c, t) for c in range(n) for t in range(n) if abs(c - t) >= 2]
    specs = []
    for layer in range(layers):
        ang = rng.uniform(0.0, 2 * np.pi, size=(n, 3))
        specs += [("U3", (q,), tuple(ang[q])) for q in range(n)]
        for a in range(layer % 2, n - 1, 2):
            specs.append(("CZ" if layer % 2 == 0 else "CX", (a, a + 1)))
            if rng.random() < p_long:
                c, t = long_pairs[int(rng.integers(len(long_pairs)))]
                specs.append(("CX", (c, t)))
    return make_gates(specs)


def brickwork_c3(n: int = 32, layers: int = 60, seed: int = 3) -> np.ndarray:
    """U3 on all qubits, then n/2 CX on a uniform random perfect matching of
    the qubits (shuffle, pair consecutive entries, first = control)."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(layers):
        ang = rng.uniform(0.0, 2 * np.pi, size=(n, 3))
        specs += [("U3", (q,), tuple(ang[q])) for q in range(n)]
        perm = rng.permutation(n)
        specs += [("CX", (int(perm[2 * j]), int(perm[2 * j + 1]))) for j in range(n // 2)]
    return make_gates(specs)


def ansatz(n: int, layers: int):
    """Hardware-efficient ansatz: per layer an RY layer, an RZ layer (both
    parameterised), then the CX ladder CX(i, i+1), i = 0..n-2.
    Returns (gates, n_params); RY on q in layer l uses parameter 2*n*l + q,
    RZ uses 2*n*l + n + q."""
    specs = []
    for layer in range(layers):
        specs += [("RY", (q,), (), 2 * n * layer + q) for q in range(n)]
        specs += [("RZ", (q,), (), 2 * n * layer + n + q) for q in range(n)]
        specs += [("CX", (i, i + 1)) for i in range(n - 1)]
    return make_gates(specs), 2 * n * layers


def ansatz_params(n_params: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-np.pi, np.pi, size=n_params)


def ansatz_batch(batch: int = 2048, n: int = 14, dmin: int = 4, dmax: int = 16, seed: int = 5):
    """``batch`` instances of the ansatz with depths iid uniform on
    {dmin..dmax}; parameters iid U[-pi, pi).  Returns (list of gate arrays,
    depths, list of theta arrays)."""
    rng = np.random.default_rng(seed)
    depths = rng.integers(dmin, dmax + 1, size=batch)
    circs, thetas = [], []
    for d in depths:
        g, npar = ansatz(n, int(d))
        circs.append(g)
        thetas.append(rng.uniform(-np.pi, np.pi, size=npar))
    return circs, depths, thetas


def random_circuit(n: int, n_gates: int, seed: int, n_params: int = 0, kinds=None):
    """Mixed random circuit over every gate kind (tests).  Parameterised
    rotations draw a parameter index in [0, n_params) when ``n_params > 0``.
    MAT1/MAT2 carry Haar-ish random unitaries (QR of a complex Gaussian)."""
    rng = np.random.default_rng(seed)
    names = kinds or (["H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY", "RZ", "P", "U3", "MAT1"]
                      + (["CX", "CY", "CZ", "CP", "SWAP", "RZZ", "MAT2"] if n >= 2 else []))
    specs = []
    for _ in range(n_gates):
        name = names[int(rng.integers(len(names)))]
        if name in ONE_QUBIT:
            qs = (int(rng.integers(n)),)
        else:
            a, b = rng.choice(n, size=2, replace=False)
            qs = (int(a), int(b))
        ang = tuple(rng.uniform(-2 * np.pi, 2 * np.pi, size=3))
        param = -1
        if name in PARAM_KINDS and n_params > 0 and rng.random() < 0.7:
            param = int(rng.integers(n_params))
        mat = None
        if name in ("MAT1", "MAT2"):
            d = 2 if name == "MAT1" else 4
            z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
            q, r = np.linalg.qr(z)
            mat = q * (np.diag(r) / np.abs(np.diag(r)))
        specs.append((name, qs, ang, param, mat))
    return make_gates(specs)


def inverse_circuit(gates: np.ndarray, theta=None) -> np.ndarray:
    """The inverse circuit: gates in reverse order, each replaced by its
    textbook inverse (S <-> SDG, T <-> TDG, SX^-1 = SX^3, rotations and phases
    with negated angle, U3(t, p, l)^-1 = U3(-t, -l, -p), MAT -> conjugate
    transpose).  Parameterised angles are resolved from ``theta``."""
    specs = []
    for g in gates[::-1]:
        name = KIND_NAME[int(g["kind"])]
        qs = (int(g["q0"]),) if name in ONE_QUBIT else (int(g["q0"]), int(g["q1"]))
        a = np.array(g["angle"], dtype=np.float64)
        if int(g["param"]) >= 0:
            a[0] = float(theta[int(g["param"])])
        if name in ("H", "X", "Y", "Z", "CX", "CY", "CZ", "SWAP"):
            specs.append((name, qs))
        elif name in ("S", "T"):
            specs.append((name + "DG", qs))
        elif name in ("SDG", "TDG"):
            specs.append((name[:-2], qs))
        elif name == "SX":
            specs += [("SX", qs)] * 3
        elif name in ("RX", "RY", "RZ", "P", "CP", "RZZ"):
            specs.append((name, qs, (-a[0],)))
        elif name == "U3":
            specs.append(("U3", qs, (-a[0], -a[2], -a[1])))
        else:
            d = 2 if name == "MAT1" else 4
            buf = np.asarray(g["mat"])[:2 * d * d]
            m = (buf[0::2] + 1j * buf[1::2]).reshape(d, d)
            specs.append((name, qs, (), -1, m.conj().T))
    return make_gates(specs)


# ---------------------------------------------------------------- observables

def pauli_sum(terms) -> np.ndarray:
    """``terms``: iterable of (coeff, {qubit: 'X'|'Y'|'Z'})."""
    out = np.zeros(len(terms), dtype=PAULI_DTYPE)
    for i, (c, ops) in enumerate(terms):
        xm = zm = 0
        for q, p in ops.items():
            if p in ("X", "Y"):
                xm |= 1 << q
            if p in ("Z", "Y"):
                zm |= 1 << q
        out[i] = (c, xm, zm)
    return out


def z_on(q: int) -> np.ndarray:
    return pauli_sum([(1.0, {q: "Z"})])


def zz_chain(n: int) -> np.ndarray:
    """sum_{i=0}^{n-2} Z_i Z_{i+1} (open chain)."""
    return pauli_sum([(1.0, {i: "Z", i + 1: "Z"}) for i in range(n - 1)])


def zz_chain_plus_x(n: int, hx: float = 0.5) -> np.ndarray:
    """sum_{i=0}^{n-2} Z_i Z_{i+1} + hx * sum_i X_i."""
    return pauli_sum([(1.0, {i: "Z", i + 1: "Z"}) for i in range(n - 1)]
                     + [(hx, {i: "X"}) for i in range(n)])


# ---------------------------------------------------------------- named workloads

WORKLOADS = {
    "c1": dict(desc="12-qubit U3+CZ brickwork, 20 layers, seed 1", n=12),
    "c2": dict(desc="28-qubit U3 + CZ/CX brickwork + 5% long-range CX, 40 layers, seed 2, k=10", n=28),
    "c3": dict(desc="32-qubit U3 + random-matching CX, 60 layers, seed 3", n=32),
    "c4": dict(desc="20-qubit RY.RZ + CX-ladder ansatz, 10 layers, 400 params, seed 4", n=20),
    "c5": dict(desc="2048 x 14-qubit ansatz, depths U{4..16}, seed 5", n=14),
}
