"""OpenQASM 2 text through the whole HIP path: qasm.parse -> qsv_partition
-> qsv_apply (table-driven and specialised sweeps) against the complex128
oracle on the same parsed gates: the paper's GHZ-3 listing (Section 4.1), the
text qasm.dump writes for the 20-qubit QFT and the 12-qubit brickwork, and a
hand-written program over every statement the reader takes, including rz in
its rotation reading."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_14098_amd as Q
from paper_2509_14098_amd import qasm
import workloads as W

pytestmark = pytest.mark.gpu

GHZ3 = """OPENQASM 2.0;
include "qelib1.inc";
qreg q[3];
creg c[3];
h q[0];
cx q[0],q[1];
cx q[1],q[2];
measure q[0] -> c[0];
"""

EVERY_STATEMENT = """OPENQASM 2.0;
include "qelib1.inc";
qreg a[5];
qreg b[4];
creg c[2];
h a[0]; x a[1]; y a[2]; z a[3]; s a[4]; sdg b[0]; t b[1]; tdg b[2]; sx b[3];
id a[0];
rx(pi/3) a[0]; ry(-0.7) a[1]; rz(2*pi/5) a[2]; p(0.25) a[3]; u1(-1.5) a[4];
u3(0.3, 1.1, -0.4) b[0]; u(1.2, 0.2, 0.9) b[1]; U(0.5, -2.0, 3.0) b[2];
barrier a[0], b[3];
cx a[0], b[3]; CX b[3], a[1]; cy a[2], b[0]; cz a[3], a[4]; cp(pi/7) b[1], a[0];
cu1(0.6) a[1], b[2]; swap a[2], b[3]; rzz(1.3) a[4], b[0];
h b[2]; rz(-(1+2)*0.1) b[1];
measure b[2] -> c[0];
"""


@pytest.fixture(scope="module")
def sim():
    s = Q.Simulator(0)
    yield s
    s.close()


def run_text(sim, text, k, specialise=False):
    n, gates = qasm.parse(text)
    plan = sim.partition(n, gates, k)
    try:
        if specialise:
            sim.specialise(plan)
        psi = sim.zero_state(n)
        sim.apply(plan, psi)
        torch.cuda.synchronize()
        return n, gates, psi.cpu().numpy()
    finally:
        plan.close()


def test_ghz3_listing_on_the_gpu(sim):
    n, gates, psi = run_text(sim, GHZ3, 2)
    ref = np.zeros(8, complex)
    ref[0] = ref[7] = 2 ** -0.5
    assert n == 3 and np.max(np.abs(psi - ref)) < 1e-7
    assert np.max(np.abs(psi - oracle.apply(n, gates))) < 1e-7


@pytest.mark.parametrize("specialise", [False, True], ids=["table", "specialised"])
@pytest.mark.parametrize("name", ["qft20", "c1"])
def test_dumped_workloads_on_the_gpu(sim, name, specialise):
    n, gates0 = (20, W.qft(20)) if name == "qft20" else (12, W.brickwork_c1())
    text = qasm.dump(n, gates0)
    n2, gates, psi = run_text(sim, text, 10 if n > 12 else 8, specialise)
    assert n2 == n and np.array_equal(gates["kind"], gates0["kind"])
    ref = oracle.apply(n, gates)
    err = float(np.max(np.abs(psi - ref)))
    print(f"{name} from OpenQASM text ({'specialised' if specialise else 'table-driven'}): max-abs {err:.2e}",
          flush=True)
    assert err < 1e-5
    if name == "qft20":  # the QFT of |0..0> is the uniform superposition
        assert np.max(np.abs(psi - 2 ** (-n / 2))) < 1e-5


@pytest.mark.parametrize("k", [4, 8])
def test_every_statement_on_the_gpu(sim, k):
    n, gates, psi = run_text(sim, EVERY_STATEMENT, k)
    assert n == 9
    ref = oracle.apply(n, gates)
    assert np.max(np.abs(psi - ref)) < 1e-6
    # rz is the rotation exp(-i a Z / 2): the same program with rz written as
    # its qelib1 form u1 differs from it by a global phase only
    n_u1, g_u1 = qasm.parse(EVERY_STATEMENT.replace("rz(2*pi/5)", "u1(2*pi/5)").replace("rz(-(1+2)*0.1)",
                                                                                        "u1(-(1+2)*0.1)"))
    ref_u1 = oracle.apply(n_u1, g_u1)
    phase = np.exp(-0.5j * (2 * np.pi / 5 - 0.3))
    assert np.max(np.abs(ref_u1 * phase - ref)) < 1e-12
