"""ctypes binding of libqsv.so: same names as the C interface (include/qsv.h).

Only argument marshalling happens here.  Device buffers are torch tensors on
the GPU (their ``data_ptr()`` is passed through); host arrays are numpy
structured arrays whose layout is the C record.  torch is imported before the
library is loaded so that the process has one HIP runtime.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # (must be loaded before libqsv.so: one HIP runtime per process)

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libqsv.so")

GATE_DTYPE = np.dtype([
    ("kind", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("param", "<i4"),
    ("angle", "<f8", (3,)), ("mat", "<f8", (32,)),
], align=True)
PAULI_DTYPE = np.dtype([("coeff", "<f8"), ("x_mask", "<u8"), ("z_mask", "<u8")], align=True)
KIND = dict(H=1, X=2, Y=3, Z=4, S=5, SDG=6, T=7, TDG=8, SX=9, RX=10, RY=11, RZ=12, P=13, U3=14,
            CX=20, CY=21, CZ=22, CP=23, SWAP=24, RZZ=25, MAT1=30, MAT2=31)
PLAN_GATE_BY_GATE = 1
PLAN_GRAD = 2
PLAN_TUNE_SPECIALISED = 4


class QsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qsv error {code}: {msg}")
        self.code = code


class _TileConfig(ctypes.Structure):
    _fields_ = [("reg_qubits", ctypes.c_int32), ("log_threads", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_circuits", ctypes.c_int32), ("k_local", ctypes.c_int32),
                ("tile_qubits", ctypes.c_int32), ("reg_qubits", ctypes.c_int32), ("log_threads", ctypes.c_int32),
                ("n_gates", ctypes.c_int64), ("n_params", ctypes.c_int64), ("n_partitions", ctypes.c_int64),
                ("n_stages", ctypes.c_int64), ("ckpt_bytes", ctypes.c_int64), ("flops_per_apply", ctypes.c_double),
                ("bytes_per_apply", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("specialise_seconds", ctypes.c_double), ("specialised", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
EXPORTS = ["qsv_last_error", "qsv_create", "qsv_destroy", "qsv_set_stream", "qsv_partition", "qsv_plan_destroy",
           "qsv_plan_get_info", "qsv_plan_params", "qsv_plan_partition", "qsv_apply", "qsv_expect",
           "qsv_expect_noalloc",
           "qsv_adjoint_grad", "qsv_set_timing", "qsv_last_sweep_ms", "qsv_last_sweep_times", "qsv_last_batch_clock", "qsv_last_autotune",
           "qsv_partition_distributed", "qsv_plan_distributed_info", "qsv_plan_specialise",
           "qsv_plan_specialise_async"]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libqsv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise QsvError(-6, f"{_LIB_PATH} is not built (run python -m paper_2509_14098_amd.build)")
    lib = ctypes.CDLL(_LIB_PATH)
    V, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.qsv_last_error.restype = ctypes.c_char_p
    sigs = {
        "qsv_create": [I32, V, V], "qsv_destroy": [V], "qsv_set_stream": [V, V],
        "qsv_partition": [V, I32, V, V, I32, I32, U32, V, V], "qsv_plan_destroy": [V],
        "qsv_plan_get_info": [V, V], "qsv_plan_specialise": [V, V, V], "qsv_plan_specialise_async": [V, V], "qsv_plan_params": [V, I32, V, V],
        "qsv_plan_partition": [V, I32, I32, I64, V, V, I64, V],
        "qsv_apply": [V, V, V, V, V], "qsv_expect": [V, V, I32, I32, I64, V, V],
        "qsv_expect_noalloc": [V, V, I32, I32, I64, V, V],
        "qsv_adjoint_grad": [V, V, V, I32, V, V, V, V, V],
        "qsv_set_timing": [V, I32], "qsv_last_sweep_ms": [V, V, V], "qsv_last_sweep_times": [V, V, I64, V], "qsv_last_batch_clock": [V, V, I64, V, V], "qsv_last_autotune": [V, I32],
        "qsv_partition_distributed": [V, I32, V, I64, I32, I32, U32, V, V],
        "qsv_plan_distributed_info": [V, V, V, V, V],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = I32
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise QsvError(rc, load_library().qsv_last_error().decode())


def _dptr(t, dtype=None, min_numel=0, name="tensor"):
    """Device address of a torch tensor (None -> NULL), after checking that it
    is a contiguous GPU tensor of the element type the C interface reads and
    holds at least min_numel elements."""
    if t is None:
        return None
    if not t.is_cuda:
        raise QsvError(-1, f"{name}: expected a GPU tensor")
    if not t.is_contiguous():
        raise QsvError(-1, f"{name}: expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise QsvError(-1, f"{name}: expected {dtype}, got {t.dtype}")
    if t.numel() < min_numel:
        raise QsvError(-1, f"{name}: {t.numel()} elements, the call needs {min_numel}")
    return ctypes.c_void_p(t.data_ptr())


def _state_len(plan):
    i = qsv_plan_info(plan)
    return i, i["n_circuits"] << i["n_qubits"]


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def qsv_create(device: int = 0, stream=None):
    h = ctypes.c_void_p()
    _check(load_library().qsv_create(device, _stream_ptr(stream), ctypes.byref(h)))
    return h


def qsv_destroy(ctx):
    _check(load_library().qsv_destroy(ctx))


def qsv_set_stream(ctx, stream):
    _check(load_library().qsv_set_stream(ctx, _stream_ptr(stream)))


def qsv_set_timing(ctx, enable: bool):
    _check(load_library().qsv_set_timing(ctx, 1 if enable else 0))


def qsv_last_sweep_ms(ctx):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load_library().qsv_last_sweep_ms(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def qsv_last_sweep_times(ctx):
    """Per-launch ms of the last qsv_apply (timing enabled), as a numpy array."""
    n = ctypes.c_int64()
    _check(load_library().qsv_last_sweep_times(ctx, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), dtype=np.float32)
    _check(load_library().qsv_last_sweep_times(ctx, out.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
    return out[:n.value]


def qsv_last_batch_clock(ctx):
    """(start, exit) clock ticks per workgroup of the last timed batched
    launch, as an (n, 2) uint64 array, and the clock rate in ticks/s."""
    n, hz = ctypes.c_int64(), ctypes.c_double()
    _check(load_library().qsv_last_batch_clock(ctx, None, 0, ctypes.byref(n), ctypes.byref(hz)))
    out = np.zeros((max(n.value, 1), 2), dtype=np.uint64)
    _check(load_library().qsv_last_batch_clock(ctx, out.ctypes.data_as(ctypes.c_void_p), 2 * n.value,
                                               ctypes.byref(n), None))
    return out[:n.value], hz.value


def qsv_partition(ctx, n_qubits: int, gates, circ_offsets=None, k_local: int = 0, flags: int = 0, tile=None):
    """gates: numpy array with the qsv_gate layout; circ_offsets: n_circuits+1
    offsets (default: one circuit).  tile: (reg_qubits, log_threads) or None."""
    g = np.ascontiguousarray(gates)
    if g.dtype.itemsize != GATE_DTYPE.itemsize:
        raise QsvError(-1, "gate records must have the qsv_gate layout")
    off = np.ascontiguousarray(np.array([0, len(g)] if circ_offsets is None else circ_offsets, dtype=np.int64))
    tc = _TileConfig(*(tile or (0, 0)))
    h = ctypes.c_void_p()
    _check(load_library().qsv_partition(ctx, n_qubits, g.ctypes.data_as(ctypes.c_void_p) if len(g) else None,
                                         off.ctypes.data_as(ctypes.c_void_p), len(off) - 1, k_local, flags,
                                         ctypes.byref(tc), ctypes.byref(h)))
    return h


def qsv_partition_distributed(ctx, n_qubits: int, gates, n_global: int, k_local: int = 0, flags: int = 0, tile=None):
    """Distributed-level plan of one circuit for 2^n_global emulated ranks."""
    g = np.ascontiguousarray(gates)
    if g.dtype.itemsize != GATE_DTYPE.itemsize:
        raise QsvError(-1, "gate records must have the qsv_gate layout")
    tc = _TileConfig(*(tile or (0, 0)))
    h = ctypes.c_void_p()
    _check(load_library().qsv_partition_distributed(ctx, n_qubits, g.ctypes.data_as(ctypes.c_void_p) if len(g) else None,
                                                    len(g), n_global, k_local, flags, ctypes.byref(tc),
                                                    ctypes.byref(h)))
    return h


def qsv_plan_distributed_info(plan) -> dict:
    ng, nd, ex, rs = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().qsv_plan_distributed_info(plan, ctypes.byref(ng), ctypes.byref(nd), ctypes.byref(ex),
                                                    ctypes.byref(rs)))
    return dict(n_global=ng.value, n_dist_partitions=nd.value, exchange_swaps=ex.value, remap_swaps=rs.value)


def qsv_last_autotune():
    """[(k, reg_qubits, log_threads, ms)] of the last autotuning run in this process."""
    n = load_library().qsv_last_autotune(None, 0)
    buf = np.zeros(4 * max(n, 1), dtype=np.int32)
    load_library().qsv_last_autotune(buf.ctypes.data_as(ctypes.c_void_p), n)
    return [(int(buf[4 * i]), int(buf[4 * i + 1]), int(buf[4 * i + 2]), buf[4 * i + 3] / 1000.0) for i in range(n)]


def qsv_plan_destroy(plan):
    _check(load_library().qsv_plan_destroy(plan))


def qsv_plan_info(plan) -> dict:
    i = _PlanInfo()
    _check(load_library().qsv_plan_get_info(plan, ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in _PlanInfo._fields_}


def qsv_plan_specialise(ctx, plan) -> float:
    """Generate, compile and (with a context) load the plan's specialised
    sweep kernels; returns the host seconds taken."""
    secs = ctypes.c_double(0.0)
    _check(load_library().qsv_plan_specialise(ctx, plan, ctypes.byref(secs)))
    return secs.value


def qsv_plan_specialise_async(ctx, plan) -> None:
    """Start compiling the plan's specialised kernels in the background;
    qsv_apply switches to them once they are ready."""
    _check(load_library().qsv_plan_specialise_async(ctx, plan))


def qsv_plan_params(plan, circuit: int = 0):
    o, c = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().qsv_plan_params(plan, circuit, ctypes.byref(o), ctypes.byref(c)))
    return o.value, c.value


def qsv_plan_partition(plan, circuit: int, level: int, p: int):
    """(local qubit list, gate indices) of partition p (level 0) or register stage p (level 1)."""
    mask, n = ctypes.c_uint64(), ctypes.c_int64()
    _check(load_library().qsv_plan_partition(plan, circuit, level, p, ctypes.byref(mask), None, 0, ctypes.byref(n)))
    buf = np.zeros(max(n.value, 1), dtype=np.int32)
    _check(load_library().qsv_plan_partition(plan, circuit, level, p, ctypes.byref(mask),
                                             buf.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
    m = mask.value
    return [q for q in range(64) if (m >> q) & 1], buf[:n.value].tolist()


def qsv_apply(ctx, plan, theta, psi, ckpt=None):
    i, dim = _state_len(plan)
    _check(load_library().qsv_apply(
        ctx, plan, _dptr(theta, torch.float64, i["n_params"], "theta"), _dptr(psi, torch.complex64, dim, "psi"),
        _dptr(ckpt, torch.complex64, i["ckpt_bytes"] // 8, "ckpt")))


def _pauli(H):
    h = np.ascontiguousarray(H)
    if len(h) and h.dtype.itemsize != PAULI_DTYPE.itemsize:
        raise QsvError(-1, "Pauli terms must have the qsv_pauli_term layout")
    return h, (h.ctypes.data_as(ctypes.c_void_p) if len(h) else None)


def qsv_expect(ctx, H, n_qubits: int, batch: int, psi, out):
    h, hp = _pauli(H)
    dim = batch << n_qubits if 0 < n_qubits < 63 and batch > 0 else 0
    _check(load_library().qsv_expect(ctx, hp, len(h), n_qubits, batch, _dptr(psi, torch.complex64, dim, "psi"),
                                     _dptr(out, torch.float64, max(batch, 0), "out")))


def qsv_expect_noalloc(ctx, H, n_qubits: int, batch: int, psi, out):
    h, hp = _pauli(H)
    dim = batch << n_qubits if 0 < n_qubits < 63 and batch > 0 else 0
    _check(load_library().qsv_expect_noalloc(ctx, hp, len(h), n_qubits, batch,
                                             _dptr(psi, torch.complex64, dim, "psi"),
                                             _dptr(out, torch.float64, max(batch, 0), "out")))


def qsv_adjoint_grad(ctx, plan, H, theta, psi_final, ckpt, energy, grad):
    h, hp = _pauli(H)
    i, dim = _state_len(plan)
    _check(load_library().qsv_adjoint_grad(
        ctx, plan, hp, len(h), _dptr(theta, torch.float64, i["n_params"], "theta"),
        _dptr(psi_final, torch.complex64, dim, "psi_final"), _dptr(ckpt, torch.complex64, i["ckpt_bytes"] // 8, "ckpt"),
        _dptr(energy, torch.float64, i["n_circuits"], "energy"), _dptr(grad, torch.float64, i["n_params"], "grad")))
