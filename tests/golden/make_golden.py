"""Write oracle-computed expected values for the large parity tests.

Runs only the complex128 oracle (oracle/) on circuits from workloads/ and
stores, per workload: the amplitudes at a seeded sample of indices, the first
1024 amplitudes, the squared norm, <Z_0> and <sum Z_i Z_i+1>.  The GPU tests
compare the GPU state at the same indices.  Nothing here reads GPU results.

    python tests/golden/make_golden.py c2 c3n24 c3n26
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    "c2": lambda: (28, W.brickwork_c2()),
    "c3n24": lambda: (24, W.brickwork_c3(n=24)),
    "c3n26": lambda: (26, W.brickwork_c3(n=26)),
}


def sample_indices(n, count=4096, seed=12345):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 1 << n, size=count, dtype=np.int64)
    return np.unique(np.concatenate([idx, np.arange(min(1024, 1 << n)), [(1 << n) - 1]]))


def make(name):
    n, gates = CASES[name]()
    t0 = time.time()
    psi = oracle.apply(n, gates)
    t1 = time.time()
    idx = sample_indices(n)
    out = dict(
        n=np.int64(n), n_gates=np.int64(len(gates)), circuit_sha256=np.bytes_(W.circuit_hash(gates, n)),
        idx=idx, amp=psi[idx], norm2=np.float64(oracle.norm2(psi)),
        z0=np.float64(oracle.expect(n, W.z_on(0), psi)),
        zz=np.float64(oracle.expect(n, W.zz_chain(n), psi)),
        oracle_seconds=np.float64(t1 - t0), oracle_threads=np.int64(oracle.threads()),
    )
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: n={n} gates={len(gates)} oracle {t1 - t0:.1f}s ({oracle.threads()} threads) -> {path}",
          flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        make(name)
