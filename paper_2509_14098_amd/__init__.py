"""qsv: partitioned state-vector simulation on AMD MI355X (gfx950).

Python binding of the C interface declared in ``include/qsv.h``.  Every call
marshals arguments and forwards them to ``libqsv.so``; all computation (graph
analysis, partitioning, the GPU sweeps, reductions and gradients) happens in
the native library.  torch provides device memory and the current stream.
There is no fallback: if the native library is missing, importing the binding
succeeds but every call raises.
"""
from .binding import (  # noqa: F401
    QsvError, GATE_DTYPE, PAULI_DTYPE, KIND, PLAN_GATE_BY_GATE, PLAN_GRAD, PLAN_TUNE_SPECIALISED,
    qsv_create, qsv_destroy, qsv_set_stream, qsv_partition, qsv_plan_destroy, qsv_plan_info,
    qsv_plan_params, qsv_plan_partition, qsv_apply, qsv_expect, qsv_expect_noalloc, qsv_adjoint_grad,
    qsv_set_timing, qsv_last_sweep_ms, qsv_last_sweep_times, qsv_last_batch_clock, qsv_last_autotune, library_path, load_library,
    qsv_partition_distributed, qsv_plan_distributed_info, qsv_plan_specialise, qsv_plan_specialise_async,
)
from .sim import Simulator, Plan, Energy  # noqa: F401
