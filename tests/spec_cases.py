"""Circuits of the specialised-kernel parity tests (tests/test_gpu_specialised.py).
The CPU suite checks that together they lower to every register-level op kind."""

# n, gates, k, (reg_qubits, log_threads): random circuits over every gate kind
# (seed 5000 + n, 5 parameters)
RANDOM_CASES = [(3, 60, 2, (3, 6)), (7, 100, 5, (4, 6)), (11, 200, 7, (4, 8)), (13, 250, 10, (5, 8)),
                (16, 300, 12, (4, 9)), (20, 300, 12, (5, 8))]

# every kernel shape whose tile fits 64 KiB of LDS (at most 13 qubits):
# (reg_qubits, log_threads) -> a circuit on reg_qubits + log_threads + 2 qubits
SHAPES = [(1, 6), (2, 6), (3, 6), (4, 6), (5, 6), (3, 8), (4, 8), (5, 8), (3, 9), (4, 9), (3, 10)]
