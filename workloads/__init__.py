"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *describes* circuits and observables (gate kinds, qubits,
angles, Pauli masks).  It holds none of the simulation arithmetic: no gate
matrices, no state updates, no partitioning.
"""
from .circuits import (  # noqa: F401
    GATE_DTYPE, PAULI_DTYPE, KIND, PARAM_KINDS, KIND_NAME,
    make_gates, circuit_hash, inverse_circuit, ghz, uniform_h, u3_layer, qft,
    brickwork_c1, brickwork_c2, brickwork_c3, ansatz, ansatz_params, ansatz_batch,
    random_circuit, pauli_sum, zz_chain_plus_x, z_on, zz_chain,
    WORKLOADS,
)
