"""ORACLE — test infrastructure only.

Plain, slow, obviously-correct CPU implementations of what the GPU path
computes, used to check it.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the product
library and its Python binding never do.  It shares no code with the GPU path.

* ``oracle.c`` (loaded here through ctypes): complex128 gate-by-gate
  simulation (paper Section 3.1, Eq. 5-6 and Eq. 9), Pauli-sum expectation
  values and the adjoint gradient.
* ``centrality.py``: the contraction graph, critical-path lengths, reachable
  sets and closeness centrality by brute force (Section 4.1, Section 4.2,
  Eq. 10-13) and the greedy frontier partitioner (Section 4.2, Fig. 5 step 3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from workloads.circuits import GATE_DTYPE, PAULI_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP over the amplitude loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_apply.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int64, P]
        lib.oracle_apply_range.argtypes = [ctypes.c_int, P, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64, P]
        lib.oracle_expect.argtypes = [ctypes.c_int, P, ctypes.c_int, P]
        lib.oracle_expect.restype = ctypes.c_double
        lib.oracle_norm2.argtypes = [ctypes.c_int, P]
        lib.oracle_norm2.restype = ctypes.c_double
        lib.oracle_adjoint.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int,
                                       P, P]
        lib.oracle_gate_matrix.argtypes = [P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _theta(theta):
    t = np.ascontiguousarray(np.zeros(1) if theta is None or len(theta) == 0 else theta, dtype=np.float64)
    return t, (0 if theta is None else len(theta))


def threads() -> int:
    return int(_load().oracle_threads())


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply(n: int, gates: np.ndarray, theta=None, psi=None) -> np.ndarray:
    """psi <- U_G ... U_1 psi (default |0...0>); complex128."""
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    psi = zero_state(n) if psi is None else np.ascontiguousarray(psi, dtype=np.complex128).copy()
    th, npar = _theta(theta)
    rc = _load().oracle_apply(n, _ptr(gates), len(gates), _ptr(th), npar, _ptr(psi))
    if rc != 0:
        raise ValueError(f"oracle_apply: invalid input (code {rc})")
    return psi


def apply_range(n: int, gates: np.ndarray, g0: int, g1: int, psi: np.ndarray, theta=None) -> None:
    """In-place application of gates[g0:g1] (used for bounded CPU timings)."""
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    th, npar = _theta(theta)
    rc = _load().oracle_apply_range(n, _ptr(gates), g0, g1, _ptr(th), npar, _ptr(psi))
    if rc != 0:
        raise ValueError(f"oracle_apply_range: invalid input (code {rc})")


def expect(n: int, H: np.ndarray, psi: np.ndarray) -> float:
    H = np.ascontiguousarray(H, dtype=PAULI_DTYPE)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return float(_load().oracle_expect(n, _ptr(H), len(H), _ptr(psi)))


def norm2(psi: np.ndarray) -> float:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(np.log2(psi.size))
    return float(_load().oracle_norm2(n, _ptr(psi)))


def adjoint(n: int, gates: np.ndarray, theta, H: np.ndarray):
    """Energy <H> and d<H>/d theta by the adjoint method; complex128."""
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    H = np.ascontiguousarray(H, dtype=PAULI_DTYPE)
    th, npar = _theta(theta)
    grad = np.zeros(max(npar, 1))
    e = ctypes.c_double(0.0)
    rc = _load().oracle_adjoint(n, _ptr(gates), len(gates), _ptr(th), npar, _ptr(H), len(H),
                                ctypes.cast(ctypes.pointer(e), ctypes.c_void_p), _ptr(grad))
    if rc != 0:
        raise ValueError(f"oracle_adjoint: invalid input (code {rc})")
    return e.value, grad[:npar]


def gate_matrix(gate, theta=None) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(gate, dtype=GATE_DTYPE).reshape(1))
    th, _ = _theta(theta)
    out = np.zeros(32)
    k = _load().oracle_gate_matrix(_ptr(g), _ptr(th), _ptr(out))
    if k == 0:
        raise ValueError("unknown gate kind")
    d = 2 if k == 1 else 4
    return (out[0:2 * d * d:2] + 1j * out[1:2 * d * d:2]).reshape(d, d)


def expect_state(n, H, psi):  # convenience alias
    return expect(n, H, psi)
