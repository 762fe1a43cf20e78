"""The lowered plans executed on the CPU (test-only emulation of the kernels'
register-level op code, tests/emu/) against the complex128 oracle: checks the
lowering — tile and stage layouts, op locations, the diagonal folding of
register stages — for every kernel shape without a GPU.  The GPU parity tests
then check the kernels themselves."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "emu", "plan_emulator.cpp")
PLANNER = os.path.join(ROOT, "paper_2509_14098_amd", "csrc", "planner.cpp")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    lib = str(tmp_path_factory.mktemp("emu") / "libplanemu.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(HERE, "emu", "shim"),
                           "-o", lib, SRC, PLANNER])
    L = ctypes.CDLL(lib)
    V = ctypes.c_void_p
    L.emu_run.argtypes = [ctypes.c_int, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int, V]
    L.emu_kind_counts.argtypes = [V, ctypes.c_int]
    L.emu_run_dist.argtypes = [ctypes.c_int, V, ctypes.c_int, V, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, V]

    def run(n, gates, k, R, LW, theta=None, flags=0, inverse=False, state=None, n_global=0):
        g = np.ascontiguousarray(gates)
        th = np.ascontiguousarray(np.zeros(1) if theta is None else theta, dtype=np.float64)
        st = np.zeros(1 << n, np.complex64)
        if state is None:
            st[0] = 1
        else:
            st[:] = state
        L.emu_run_dist(n, g.ctypes.data_as(V), len(g), th.ctypes.data_as(V), 0 if theta is None else len(theta), k,
                       R, LW, flags, int(inverse), n_global, st.ctypes.data_as(V))
        return st

    def kind_counts(reset=True):
        out = np.zeros(32, dtype=np.int64)
        L.emu_kind_counts(out.ctypes.data_as(V), int(reset))
        return out
    run.kind_counts = kind_counts
    return run


SHAPES = [(1, 6), (2, 6), (3, 6), (4, 6), (5, 6), (3, 8), (4, 8), (5, 8), (3, 9), (4, 9), (5, 9), (3, 10), (4, 10)]


@pytest.mark.parametrize("R,LW", SHAPES)
def test_random_circuits_every_shape(emu, R, LW):
    for n in (2, 5, 9, 13, 15):
        if n < 2:
            continue
        theta = np.random.default_rng(n).uniform(-3, 3, size=4)
        gates = W.random_circuit(n, 120, seed=40 + n + R, n_params=4)
        k = min(n, R + LW - 1, 9)
        out = emu(n, gates, k, R, LW, theta)
        assert np.max(np.abs(out - oracle.apply(n, gates, theta))) < 1e-5, (n, R, LW)


@pytest.mark.parametrize("name,n,gen", [("c1", 12, W.brickwork_c1),
                                        ("c2-16", 16, lambda: W.brickwork_c2(n=16, layers=12)),
                                        ("c3-16", 16, lambda: W.brickwork_c3(n=16, layers=12)),
                                        ("qft-15", 15, lambda: W.qft(15))])
def test_benchmark_shapes(emu, name, n, gen):
    gates = gen()
    ref = oracle.apply(n, gates)
    for R, LW, k in ((4, 8, 10), (5, 8, 10), (4, 9, 12)):
        assert np.max(np.abs(emu(n, gates, k, R, LW) - ref)) < 1e-5, (name, R, LW)


def test_inverse_walk_returns_to_start(emu):
    """The conjugate-transpose walk (used by the adjoint) undoes the forward plan."""
    n = 14
    theta = np.random.default_rng(3).uniform(-3, 3, size=6)
    gates = W.random_circuit(n, 200, seed=11, n_params=6)
    fwd = emu(n, gates, 10, 4, 8, theta)
    back = emu(n, gates, 10, 4, 8, theta, inverse=True, state=fwd)
    assert abs(back[0] - 1) < 1e-5 and np.max(np.abs(back[1:])) < 1e-5


def test_gate_by_gate_plan(emu):
    n = 11
    gates = W.random_circuit(n, 80, seed=5)
    assert np.max(np.abs(emu(n, gates, 8, 4, 6, flags=1) - oracle.apply(n, gates))) < 1e-5


# op kinds of the lowered plans (csrc/plan.h OpKind)
OP_KINDS = dict(U1=1, R1=2, D1=3, CX=4, CU=5, CZ=6, D2=7, U2=8, SWAP=9, DREG=10, LAYER=11, CZ_RT=12, CZ_TT=13,
                CX_T=14, D1_T=15, D2_RT=16, D2_TT=17)


def test_every_op_kind_is_exercised(emu):
    """The random circuits, fused and gate by gate, lower to every op kind the
    kernels implement, so the emulation tests above cover each code path."""
    emu.kind_counts(reset=True)
    for R, LW in ((4, 8), (3, 6), (5, 8)):
        for n in (9, 13):
            theta = np.random.default_rng(n).uniform(-3, 3, size=4)
            gates = W.random_circuit(n, 150, seed=70 + n + R, n_params=4)
            ref = oracle.apply(n, gates, theta)
            for flags in (0, 1):
                out = emu(n, gates, min(n, R + LW - 1, 9), R, LW, theta, flags=flags)
                assert np.max(np.abs(out - ref)) < 1e-5, (R, LW, n, flags)
    counts = emu.kind_counts(reset=True)
    missing = [k for k, v in OP_KINDS.items() if counts[v] == 0]
    assert not missing, missing


def test_specialised_parity_cases_cover_every_op_kind(emu):
    """The random circuits of the specialised-kernel GPU tests lower to every
    op kind as well (their plans are the ones emulated here), and the
    emulated plans match the oracle."""
    from spec_cases import RANDOM_CASES
    emu.kind_counts(reset=True)
    for n, ng, k, (R, LW) in RANDOM_CASES:
        theta = np.random.default_rng(n).uniform(-3, 3, size=5)
        gates = W.random_circuit(n, ng, seed=5000 + n, n_params=5)
        out = emu(n, gates, k, R, LW, theta)
        assert np.max(np.abs(out - oracle.apply(n, gates, theta))) < 1e-5, (n, R, LW)
    counts = emu.kind_counts(reset=True)
    missing = [k for k, v in OP_KINDS.items() if counts[v] == 0]
    assert not missing, missing


@pytest.mark.parametrize("n,g,R,LW,k", [(9, 2, 1, 6, 6), (10, 3, 1, 6, 5), (12, 4, 2, 6, 7), (14, 2, 4, 8, 10)])
def test_distributed_plans(emu, n, g, R, LW, k):
    """Distributed level: remap SWAPs between distributed partitions, each
    partition's tiles inside one rank; the final state (back in logical order)
    equals the oracle's, for random circuits, the QFT and the inverse walk."""
    theta = np.random.default_rng(n).uniform(-3, 3, size=4)
    gates = W.random_circuit(n, 160, seed=900 + n + g, n_params=4)
    ref = oracle.apply(n, gates, theta)
    out = emu(n, gates, k, R, LW, theta, n_global=g)
    assert np.max(np.abs(out - ref)) < 1e-5
    back = emu(n, gates, k, R, LW, theta, inverse=True, state=out, n_global=g)
    assert abs(back[0] - 1) < 1e-5 and np.max(np.abs(back[1:])) < 1e-5
    q = W.qft(n)
    x = (3 << n) // 7
    psi = np.zeros(1 << n, complex)
    psi[x] = 1
    out = emu(n, q, k, R, LW, state=psi, n_global=g)
    refq = np.exp(2j * np.pi * x * np.arange(1 << n) / (1 << n)) / np.sqrt(1 << n)
    assert np.max(np.abs(out - refq)) < 1e-5


@pytest.mark.parametrize("R,LW", [(4, 8), (2, 6)])
def test_parameterised_rotations_large_angles(emu, R, LW):
    """Parameterised rotations with angles spanning (-2 pi, 2 pi), forward and
    conjugate walk."""
    n = 11
    theta = np.linspace(-6.2, 6.2, 8)
    gates = W.random_circuit(n, 200, seed=31 + R, n_params=8, kinds=["RY", "RZ", "RX", "H", "CX", "CZ", "U3"])
    ref = oracle.apply(n, gates, theta)
    out = emu(n, gates, 8, R, LW, theta)
    assert np.max(np.abs(out - ref)) < 1e-5
    back = emu(n, gates, 8, R, LW, theta, inverse=True, state=out)
    assert abs(back[0] - 1) < 1e-5 and np.max(np.abs(back[1:])) < 1e-5


def test_parameterised_rz_rotations_fold_into_register_diagonals(emu):
    """The ansatz's RZ rotations on register slots fold into register
    diagonals formed from theta (OP_DREG ops, fewer than the RZ gates), and
    the plan still gives the oracle's state for random angles."""
    n, layers = 12, 3
    gates, npar = W.ansatz(n, layers)
    theta = np.random.default_rng(8).uniform(-np.pi, np.pi, size=npar)
    emu.kind_counts(reset=True)
    out = emu(n, gates, n, 4, 8, theta)
    counts = emu.kind_counts(reset=True)
    n_rz = n * layers
    assert counts[OP_KINDS["DREG"]] > 0
    assert counts[OP_KINDS["D1"]] + counts[OP_KINDS["D1_T"]] < n_rz
    assert np.max(np.abs(out - oracle.apply(n, gates, theta))) < 1e-5
