"""qsv_expect_noalloc (the entry point that allocates nothing) against
qsv_expect through the C interface: the same kernels on the same inputs give
the same float64 results bit for bit, on two calls in a row (the second with
a smaller state, batch and Pauli sum, so stale scratch contents from the
first would show), and both agree with the complex128 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_14098_amd as Q
import workloads as W

pytestmark = pytest.mark.gpu


def random_pauli_sum(n, n_terms, seed):
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_terms):
        qs = rng.choice(n, size=int(rng.integers(1, min(n, 4) + 1)), replace=False)
        terms.append((float(rng.normal()), {int(q): "XYZ"[int(rng.integers(3))] for q in qs}))
    return W.pauli_sum(terms)


def random_states(n, batch, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(batch, 1 << n)) + 1j * rng.normal(size=(batch, 1 << n))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.complex64)


@pytest.fixture(scope="module")
def sim():
    s = Q.Simulator(0)
    yield s
    s.close()


def both(sim, H, n, states):
    batch = states.shape[0]
    psi = torch.as_tensor(states, device="cuda").contiguous()
    a = torch.full((batch,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((batch,), float("nan"), dtype=torch.float64, device="cuda")
    Q.qsv_expect(sim.ctx, H, n, batch, psi, a)
    Q.qsv_expect_noalloc(sim.ctx, H, n, batch, psi, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_expect_matches_qsv_expect_twice(sim):
    # first call: 18 qubits, batch 3, 60 X/Y/Z terms (many X masks)
    n1, H1, s1 = 18, random_pauli_sum(18, 60, 1), random_states(18, 3, 2)
    print(f"noalloc call 1: n={n1} batch=3 terms={len(H1)}", flush=True)
    a1, b1 = both(sim, H1, n1, s1)
    assert np.array_equal(a1, b1), (a1, b1)
    # second call, smaller everywhere: 9 qubits, batch 1, 5 terms
    n2, H2, s2 = 9, random_pauli_sum(9, 5, 3), random_states(9, 1, 4)
    print(f"noalloc call 2: n={n2} batch=1 terms={len(H2)}", flush=True)
    a2, b2 = both(sim, H2, n2, s2)
    assert np.array_equal(a2, b2), (a2, b2)
    for H, n, s, got in ((H1, n1, s1, b1), (H2, n2, s2, b2)):
        for i in range(s.shape[0]):
            ref = oracle.expect(n, H, s[i].astype(np.complex128))
            assert abs(got[i] - ref) < 1e-9 * max(1.0, float(np.sum(np.abs(H["coeff"])))), (n, i, got[i], ref)


def test_noalloc_expect_empty_sum_and_norm(sim):
    s = random_states(12, 2, 5)
    a, b = both(sim, W.pauli_sum([]), 12, s)
    assert np.array_equal(a, b) and np.all(b == 0.0)
    a, b = both(sim, W.pauli_sum([(1.0, {})]), 12, s)
    assert np.array_equal(a, b) and np.allclose(b, 1.0, atol=1e-6)


def test_noalloc_expect_rejects_beyond_its_scratch(sim):
    psi = torch.zeros(1 << 20, dtype=torch.complex64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    too_many = W.pauli_sum([(1.0, {0: "Z"})] * 4097)
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_expect_noalloc(sim.ctx, too_many, 20, 1, psi, out)
    assert "4096" in str(e.value)
    # 300 X strings on 8 distinct qubits above qubit 3 each: every one needs a
    # 12-qubit tile pass of its own, so 300 passes x 256 blocks x batch 8 of
    # float64 partial sums (4.9 MB) exceed the 3.5 MiB the scratch holds
    rng = np.random.default_rng(9)
    highs = set()
    while len(highs) < 300:
        highs.add(tuple(sorted(rng.choice(np.arange(4, 20), size=8, replace=False).tolist())))
    wide = W.pauli_sum([(1.0, {int(q): "X" for q in h}) for h in sorted(highs)])
    psi8 = torch.zeros((8, 1 << 20), dtype=torch.complex64, device="cuda")
    out8 = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QsvError) as e:
        Q.qsv_expect_noalloc(sim.ctx, wide, 20, 8, psi8, out8)
    assert "scratch" in str(e.value)
    Q.qsv_expect_noalloc(sim.ctx, wide, 20, 1, psi8[0], out8[:1])  # 600 KiB: within the scratch
    torch.cuda.synchronize()
    assert float(out8[0]) == 0.0 and float(out[0]) == 0.0
