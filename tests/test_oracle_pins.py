"""Pins of the complex128 oracle against facts that do not come from its own
code: the paper's worked example (Section 4.1 listing: GHZ-3), closed forms,
invariants, textbook gate identities, matrix exponentials from scipy, the dense
Kronecker embedding of Eq. 5-6, a numpy tensordot version of Eq. 9 and
parameter-shift derivatives."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]])
Z = np.diag([1.0 + 0j, -1.0])
I2 = np.eye(2, dtype=complex)


def one(name, q=0, angles=(), param=-1, mat=None):
    return W.make_gates([(name, (q,), angles, param, mat)])[0]


def two(name, a, b, angles=()):
    return W.make_gates([(name, (a, b), angles)])[0]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [3, 5, 10])
def test_ghz_closed_form(n):
    # n = 3 is the paper's driving example: h q[0]; cx q[0],q[1]; cx q[1],q[2]
    psi = oracle.apply(n, W.ghz(n))
    ref = np.zeros(1 << n, complex)
    ref[0] = ref[-1] = 1 / np.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n", [1, 4, 9])
def test_uniform_superposition(n):
    psi = oracle.apply(n, W.uniform_h(n))
    assert np.max(np.abs(psi - 2 ** (-n / 2))) < 1e-15


@pytest.mark.parametrize("n", [1, 6, 11])
def test_u3_layer_product_state(n):
    gates, ang = W.u3_layer(n, seed=11 + n)
    psi = oracle.apply(n, gates)
    x = np.arange(1 << n)
    ref = np.ones(1 << n, complex)
    for q in range(n):
        b = (x >> q) & 1
        t, p = ang[q, 0], ang[q, 1]
        ref *= np.where(b == 0, np.cos(t / 2), np.exp(1j * p) * np.sin(t / 2))
    assert np.max(np.abs(psi - ref)) < 1e-14
    for q in range(n):
        assert abs(oracle.expect(n, W.z_on(q), psi) - np.cos(ang[q, 0])) < 1e-13
    if n > 1:
        zz = oracle.expect(n, W.zz_chain(n), psi)
        assert abs(zz - sum(np.cos(ang[i, 0]) * np.cos(ang[i + 1, 0]) for i in range(n - 1))) < 1e-12


# ---------------------------------------------------------------- gate definitions

ANG = 0.7312


@pytest.mark.parametrize("name", ["RX", "RY", "RZ"])
def test_rotations_are_matrix_exponentials(name):
    P = {"RX": X, "RY": Y, "RZ": Z}[name]
    for a in (ANG, -2.1, 3.9):
        m = oracle.gate_matrix(one(name, angles=(a,)))
        assert np.max(np.abs(m - sla.expm(-0.5j * a * P))) < 1e-14


def test_rzz_is_matrix_exponential():
    m = oracle.gate_matrix(two("RZZ", 0, 1, (ANG,)))
    assert np.max(np.abs(m - sla.expm(-0.5j * ANG * np.kron(Z, Z)))) < 1e-14


def test_u3_euler_form():
    # OpenQASM 2: U3(t, p, l) = e^{i(p+l)/2} RZ(p) RY(t) RZ(l)
    t, p, l = 1.1, -0.4, 2.3
    m = oracle.gate_matrix(one("U3", angles=(t, p, l)))
    rz = lambda a: sla.expm(-0.5j * a * Z)
    ry = sla.expm(-0.5j * t * Y)
    assert np.max(np.abs(m - np.exp(0.5j * (p + l)) * rz(p) @ ry @ rz(l))) < 1e-14


def test_fixed_gate_identities():
    gm = lambda name, **kw: oracle.gate_matrix(one(name, **kw))
    H, Xo, Yo, Zo = gm("H"), gm("X"), gm("Y"), gm("Z")
    assert np.allclose(H @ Zo @ H, Xo, atol=1e-15) and np.allclose(H @ Xo @ H, Zo, atol=1e-15)
    assert np.allclose(Xo, X) and np.allclose(Yo, 1j * X @ Z)
    S, T, SX = gm("S"), gm("T"), gm("SX")
    assert np.allclose(S @ S, Zo) and np.allclose(T @ T, S) and np.allclose(SX @ SX, Xo)
    assert np.allclose(gm("SDG"), S.conj().T) and np.allclose(gm("TDG"), T.conj().T)
    assert np.allclose(gm("U3", angles=(ANG, -np.pi / 2, np.pi / 2)), gm("RX", angles=(ANG,)))
    assert np.allclose(gm("U3", angles=(ANG, 0, 0)), gm("RY", angles=(ANG,)))
    assert np.allclose(gm("U3", angles=(0, 0, ANG)), gm("P", angles=(ANG,)))
    assert np.allclose(gm("RZ", angles=(ANG,)), np.exp(-0.5j * ANG) * gm("P", angles=(ANG,)))


@pytest.mark.parametrize("name", list(W.KIND))
def test_every_gate_unitary(name):
    rng = np.random.default_rng(7)
    g = W.random_circuit(3, 1, seed=3, kinds=[name])[0]
    m = oracle.gate_matrix(g, rng.uniform(-3, 3, size=4))
    assert np.max(np.abs(m.conj().T @ m - np.eye(len(m)))) < 1e-14


def _state_after(n, specs, psi0):
    return oracle.apply(n, W.make_gates(specs), psi=psi0)


def test_two_qubit_gate_identities_on_states():
    """CZ = H_t CX H_t; SWAP = CX CX' CX; RZZ = CX RZ_t CX; CY = S_t CX S_t^dag;
    CX flips the target exactly when the control is 1 (paper Fig. 1b)."""
    n = 4
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=16) + 1j * rng.normal(size=16)
    psi0 /= np.linalg.norm(psi0)
    for c, t in ((0, 1), (3, 1), (2, 0)):
        eq = lambda a, b: np.max(np.abs(_state_after(n, a, psi0) - _state_after(n, b, psi0))) < 1e-14
        assert eq([("CZ", (c, t))], [("H", (t,)), ("CX", (c, t)), ("H", (t,))])
        assert eq([("SWAP", (c, t))], [("CX", (c, t)), ("CX", (t, c)), ("CX", (c, t))])
        assert eq([("RZZ", (c, t), (ANG,))], [("CX", (c, t)), ("RZ", (t,), (ANG,)), ("CX", (c, t))])
        assert eq([("CY", (c, t))], [("SDG", (t,)), ("CX", (c, t)), ("S", (t,))])
        assert eq([("CP", (c, t), (ANG,))], [("CP", (t, c), (ANG,))])
        out = _state_after(n, [("CX", (c, t))], psi0)
        x = np.arange(16)
        src = np.where((x >> c) & 1, x ^ (1 << t), x)
        assert np.max(np.abs(out - psi0[src])) < 1e-15


# ---------------------------------------------------------------- Eq. 5-6 and Eq. 9 brute force

def _embed(n, g, theta):
    """Dense 2^n x 2^n operator of one gate, written from the definition of the
    Kronecker embedding (Eq. 5-6) with qubit q = bit q."""
    m = oracle.gate_matrix(g, theta)
    if len(m) == 2:
        q = int(g["q0"])
        return np.kron(np.kron(np.eye(1 << (n - 1 - q)), m), np.eye(1 << q))
    q0, q1 = int(g["q0"]), int(g["q1"])
    D = np.zeros((1 << n, 1 << n), complex)
    rest = ~((1 << q0) | (1 << q1))
    for xo in range(1 << n):
        for xi in range(1 << n):
            if (xo & rest) == (xi & rest):
                jo = ((xo >> q0) & 1) + 2 * ((xo >> q1) & 1)
                ji = ((xi >> q0) & 1) + 2 * ((xi >> q1) & 1)
                D[xo, xi] = m[jo, ji]
    return D


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (3, 3), (5, 4), (6, 5)])
def test_dense_kronecker_bruteforce(n, seed):
    theta = np.random.default_rng(seed).uniform(-3, 3, size=5)
    gates = W.random_circuit(n, 25, seed=seed, n_params=5)
    U = np.eye(1 << n, dtype=complex)
    for g in gates:
        U = _embed(n, g, theta) @ U
    assert np.max(np.abs(U.conj().T @ U - np.eye(1 << n))) < 1e-12
    psi = oracle.apply(n, gates, theta)
    assert np.max(np.abs(psi - U[:, 0])) < 1e-13


@pytest.mark.parametrize("n,seed", [(4, 8), (9, 9), (12, 10)])
def test_tensordot_contraction(n, seed):
    """Eq. 9 with numpy: the state is an n-axis tensor (axis n-1-q = qubit q in
    C order) contracted with each gate tensor."""
    theta = np.random.default_rng(seed).uniform(-3, 3, size=6)
    gates = W.random_circuit(n, 60, seed=seed, n_params=6)
    T = np.zeros((2,) * n, complex)
    T[(0,) * n] = 1
    for g in gates:
        m = oracle.gate_matrix(g, theta)
        if len(m) == 2:
            ax = n - 1 - int(g["q0"])
            T = np.moveaxis(np.tensordot(m, T, axes=([1], [ax])), 0, ax)
        else:
            a0, a1 = n - 1 - int(g["q0"]), n - 1 - int(g["q1"])
            m4 = m.reshape(2, 2, 2, 2)  # [b1_out, b0_out, b1_in, b0_in]
            T = np.tensordot(m4, T, axes=([2, 3], [a1, a0]))
            T = np.moveaxis(T, [0, 1], [a1, a0])
    psi = oracle.apply(n, gates, theta)
    assert np.max(np.abs(psi - T.reshape(-1))) < 1e-13


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("n,seed", [(3, 21), (8, 22), (13, 23)])
def test_norm_preserved_after_every_gate(n, seed):
    theta = np.random.default_rng(seed).uniform(-3, 3, size=4)
    gates = W.random_circuit(n, 80, seed=seed, n_params=4)
    psi = oracle.zero_state(n)
    for i in range(len(gates)):
        oracle.apply_range(n, gates, i, i + 1, psi, theta)
        assert abs(oracle.norm2(psi) - 1) < 1e-12


@pytest.mark.parametrize("n,seed", [(2, 31), (7, 32), (14, 33)])
def test_circuit_then_inverse_is_identity(n, seed):
    theta = np.random.default_rng(seed).uniform(-3, 3, size=4)
    gates = W.random_circuit(n, 120, seed=seed, n_params=4)
    both = np.concatenate([gates, W.inverse_circuit(gates, theta)])
    psi = oracle.apply(n, both, theta)
    assert abs(psi[0] - 1) < 1e-12 and np.max(np.abs(psi[1:])) < 1e-12


def test_brickwork_c1_inverse_and_norm():
    g = W.brickwork_c1()
    assert len(g) == 350
    psi = oracle.apply(12, g)
    assert abs(oracle.norm2(psi) - 1) < 1e-13
    back = oracle.apply(12, W.inverse_circuit(g), psi=psi)
    assert abs(back[0] - 1) < 1e-12


# ---------------------------------------------------------------- expectation values

def test_expectation_closed_forms():
    for n in (3, 6):
        ghz = oracle.apply(n, W.ghz(n))
        assert abs(oracle.expect(n, W.zz_chain(n), ghz) - (n - 1)) < 1e-14
        for i in range(n):
            assert abs(oracle.expect(n, W.pauli_sum([(1.0, {i: "X"})]), ghz)) < 1e-15
        plus = oracle.apply(n, W.uniform_h(n))
        assert abs(oracle.expect(n, W.zz_chain(n), plus)) < 1e-14
        assert abs(oracle.expect(n, W.pauli_sum([(1.0, {i: "X"}) for i in range(n)]), plus) - n) < 1e-13
    # S H |0> = (|0> + i|1>)/sqrt2 is the +1 eigenstate of Y
    y = oracle.apply(1, W.make_gates([("H", (0,)), ("S", (0,))]))
    assert abs(oracle.expect(1, W.pauli_sum([(1.0, {0: "Y"})]), y) - 1) < 1e-15


def test_zz_chain_popcount_identity():
    n = 9
    rng = np.random.default_rng(3)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    x = np.arange(1 << n)
    pc = np.array([bin(v).count("1") for v in (x ^ (x >> 1)) & ((1 << (n - 1)) - 1)])
    ref = np.sum(np.abs(psi) ** 2 * ((n - 1) - 2 * pc))
    assert abs(oracle.expect(n, W.zz_chain(n), psi) - ref) < 1e-10


@pytest.mark.parametrize("n,seed", [(2, 1), (4, 2), (6, 3)])
def test_expectation_dense_pauli_bruteforce(n, seed):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    terms = []
    for _ in range(6):
        ops = {q: "XYZ"[int(rng.integers(3))] for q in rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)}
        terms.append((float(rng.normal()), {int(k): v for k, v in ops.items()}))
    H = W.pauli_sum(terms)
    dense = np.zeros((1 << n, 1 << n), complex)
    for c, ops in terms:
        M = np.eye(1, dtype=complex)
        for q in reversed(range(n)):  # kron order: highest qubit first
            M = np.kron(M, {"X": X, "Y": Y, "Z": Z}.get(ops.get(q), I2))
        dense += c * M
    ref = np.real(np.vdot(psi, dense @ psi))
    assert abs(oracle.expect(n, H, psi) - ref) < 1e-11


# ---------------------------------------------------------------- gradients

def test_gradient_single_rotation_closed_form():
    for t in (0.3, -2.2, 1.5707):
        g = W.make_gates([("RY", (0,), (), 0)])
        e, gr = oracle.adjoint(1, g, np.array([t]), W.z_on(0))
        assert abs(e - np.cos(t)) < 1e-15 and abs(gr[0] + np.sin(t)) < 1e-15


def _energy(n, gates, theta, H):
    return oracle.expect(n, H, oracle.apply(n, gates, theta))


@pytest.mark.parametrize("n,seed", [(3, 41), (6, 42)])
def test_adjoint_equals_parameter_shift(n, seed):
    """Every parameter used by exactly one Pauli rotation: the two-point shift
    rule is exact.  Parameters used by several gates: shift each occurrence."""
    rng = np.random.default_rng(seed)
    npar = 5
    gates = W.random_circuit(n, 40, seed=seed, n_params=npar)
    theta = rng.uniform(-3, 3, size=npar)
    H = W.zz_chain_plus_x(n, 0.7)
    e, grad = oracle.adjoint(n, gates, theta, H)
    assert abs(e - _energy(n, gates, theta, H)) < 1e-12
    ref = np.zeros(npar)
    for i, g in enumerate(gates):
        p = int(g["param"])
        if p < 0:
            continue
        for s in (+1, -1):
            gg = gates.copy()
            gg[i]["param"] = -1
            gg[i]["angle"][0] = theta[p] + s * np.pi / 2
            ref[p] += s * 0.5 * _energy(n, gg, theta, H)
    assert np.max(np.abs(grad - ref)) < 1e-11


def test_central_fd_matches_sinc_bias():
    """With each parameter used once, E(theta_j) = A + R cos(theta_j - t0), so
    the central difference equals E'(theta) sin(h)/h exactly."""
    n = 5
    gates, npar = W.ansatz(n, 3)
    theta = W.ansatz_params(npar, seed=4)
    H = W.zz_chain_plus_x(n)
    e, grad = oracle.adjoint(n, gates, theta, H)
    h = 1e-3
    for j in (0, 7, npar - 1):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (_energy(n, gates, tp, H) - _energy(n, gates, tm, H)) / (2 * h)
        assert abs(fd - grad[j] * np.sin(h) / h) < 1e-10


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_qft_of_basis_states_closed_form(n):
    """The textbook QFT circuit (H, controlled phases, SWAPs) maps |x> to
    2^(-n/2) sum_y exp(2 pi i x y / 2^n) |y>: pins the oracle's H, CP and SWAP
    at many angles and the workload generator's bit order."""
    N = 1 << n
    gates = W.qft(n)
    for x in sorted({0, 1, N - 1, N // 3}):
        psi = np.zeros(N, complex)
        psi[x] = 1
        out = oracle.apply(n, gates, None, psi)
        ref = np.exp(2j * np.pi * x * np.arange(N) / N) / np.sqrt(N)
        assert np.max(np.abs(out - ref)) < 1e-12, x
