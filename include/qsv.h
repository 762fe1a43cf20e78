/*
 * qsv — partitioned state-vector simulation on AMD MI355X (gfx950).
 *
 * C interface of the library.  It implements the hot path of "A Closeness
 * Centrality-based Circuit Partitioner for Quantum Simulations"
 * (arXiv:2509.14098):
 *   - a circuit is a qubit count plus a flat ordered list of gates on given
 *     qubits (paper Section 4.1);
 *   - a p-qubit gate is a 2^p x 2^p unitary, i.e. a 2p-dimensional tensor of
 *     extent 2 (Section 3.1, Eq. 8);
 *   - a state of n qubits is 2^n complex amplitudes, i.e. an n-dimensional
 *     tensor of extent 2 (Section 3.1, Eq. 7); qubit q is bit q of the
 *     amplitude index (column-major stacking, Eq. 4);
 *   - the planner builds the contraction graph, scores every gate by closeness
 *     centrality and cuts the circuit into partitions of at most k local
 *     qubits (Section 4.2, Eq. 10-13, Fig. 5), recursively for the register
 *     level; each partition is then applied on the GPU as one fused sweep over
 *     the amplitudes (Section 4.3).
 * Expectation values, the adjoint gradient and batching are additions of this
 * library; the paper has none of them.
 *
 * Conventions of every entry point:
 *   - the return value is QSV_OK (0) or a negative qsv_status; on error
 *     qsv_last_error() returns a message (thread-local) and no device work has
 *     been queued, so outputs are untouched;
 *   - device pointers are plain HIP device addresses owned by the caller
 *     (e.g. torch tensors); host pointers are read during the call only;
 *   - device work is queued on the context's stream and is asynchronous:
 *     outputs are valid after the stream is synchronised;
 *   - state vectors are complex64: interleaved (re, im) float pairs, 8 bytes
 *     per amplitude, 2^n amplitudes per state, batches stored back to back.
 */
#ifndef QSV_PUBLIC_API_H_
#define QSV_PUBLIC_API_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qsv_status;
#define QSV_OK 0
#define QSV_E_ARG (-1)         /* invalid argument (null pointer, bad qubit, bad size) */
#define QSV_E_RANGE (-2)       /* parameter index out of range / not a rotation */
#define QSV_E_NOMEM (-3)       /* device or host allocation failed */
#define QSV_E_DEVICE (-4)      /* HIP runtime error */
#define QSV_E_STATE (-5)       /* call not valid for this plan (e.g. no gradient support) */
#define QSV_E_UNSUPPORTED (-6) /* valid request outside what this build implements */

/* Gate kinds: textbook / OpenQASM 2 definitions. */
enum {
    QSV_H = 1, QSV_X = 2, QSV_Y = 3, QSV_Z = 4, QSV_S = 5, QSV_SDG = 6, QSV_T = 7, QSV_TDG = 8, QSV_SX = 9,
    QSV_RX = 10,  /* exp(-i a X / 2) */
    QSV_RY = 11,  /* exp(-i a Y / 2) */
    QSV_RZ = 12,  /* exp(-i a Z / 2) */
    QSV_P = 13,   /* diag(1, e^{i a}) */
    QSV_U3 = 14,  /* [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]] */
    QSV_CX = 20, QSV_CY = 21, QSV_CZ = 22,
    QSV_CP = 23,  /* diag(1, 1, 1, e^{i a}) */
    QSV_SWAP = 24,
    QSV_RZZ = 25, /* exp(-i a Z(x)Z / 2) */
    QSV_MAT1 = 30, /* user 2x2 unitary in mat[0..7] */
    QSV_MAT2 = 31  /* user 4x4 unitary in mat[0..31] */
};

/*
 * One gate (296 bytes).  q0 is the target of a one-qubit gate and the control
 * of CX/CY/CZ/CP (q1 the target); SWAP/RZZ/MAT2 act on (q0, q1), MAT2 on the
 * local index j = b(q0) + 2 b(q1).  param >= 0 (RX, RY, RZ, RZZ only) takes
 * the angle from theta[param] of the gate's circuit; otherwise angle[0] (U3:
 * angle[0..2] = theta, phi, lambda).  mat holds MAT1/MAT2 matrices row-major
 * as (re, im) pairs.
 */
typedef struct qsv_gate {
    int32_t kind;
    int32_t q0;
    int32_t q1;
    int32_t param;
    double angle[3];
    double mat[32];
} qsv_gate;

/* One Pauli string with a real weight: bit q of x_mask is set for X or Y on
 * qubit q, bit q of z_mask for Z or Y. */
typedef struct qsv_pauli_term {
    double coeff;
    uint64_t x_mask;
    uint64_t z_mask;
} qsv_pauli_term;

typedef struct qsv_ctx qsv_ctx;
typedef struct qsv_plan qsv_plan;

/* Plan flags. */
#define QSV_PLAN_GATE_BY_GATE 1u /* one gate per partition: the unfused baseline, same kernels */
#define QSV_PLAN_GRAD 2u         /* keep what qsv_adjoint_grad needs (checkpoint layout) */
/* Autotune for specialised kernels (qsv_plan_specialise): candidates are timed
 * as specialised sweeps (their sampled partitions compiled, in seconds of host
 * time each), only tile shapes of at most 13 qubits are tried, and with
 * k_local > 0 only the tile shape is tuned, at that k.  Needs a context and a
 * single circuit; ignored when a tile shape is given. */
#define QSV_PLAN_TUNE_SPECIALISED 4u

/* Kernel tile shape: a workgroup of 2^log_threads threads holds a tile of
 * 2^(reg_qubits + log_threads) amplitudes, reg_qubits of them per thread.
 * All zero = library default. */
typedef struct qsv_tile_config {
    int32_t reg_qubits;  /* 1..5 */
    int32_t log_threads; /* 6..10 */
} qsv_tile_config;

typedef struct qsv_plan_info {
    int32_t n_qubits;
    int32_t n_circuits;
    int32_t k_local;         /* partition size in qubits actually used */
    int32_t tile_qubits;     /* qubits per on-chip tile */
    int32_t reg_qubits;
    int32_t log_threads;
    int64_t n_gates;         /* gates in the plan (distributed plans: with the remap SWAPs) */
    int64_t n_params;        /* total theta entries over all circuits */
    int64_t n_partitions;    /* total over circuits */
    int64_t n_stages;        /* register-level stages, total */
    int64_t ckpt_bytes;      /* size of the checkpoint buffer qsv_apply may fill */
    double flops_per_apply;  /* algorithmic flops of one qsv_apply */
    double bytes_per_apply;  /* algorithmic HBM bytes of one qsv_apply (16 B/amplitude/sweep) */
    double plan_seconds;     /* host time spent in qsv_partition */
    double specialise_seconds; /* host time of qsv_plan_specialise (compile and load), 0 if not specialised */
    int32_t specialised;     /* 1 once qsv_plan_specialise has loaded kernels for this plan */
    int32_t reserved;
} qsv_plan_info;

/* Last error message of the calling thread ("" if none). */
const char *qsv_last_error(void);

/*
 * Bind a context to a HIP device and stream (stream may be NULL = the null
 * stream of that device).  The context owns scratch memory (reduction
 * partials, the adjoint's lambda state) and is freed by qsv_destroy.
 * Errors: QSV_E_ARG (out null), QSV_E_DEVICE (no such device).
 */
qsv_status qsv_create(int32_t device, void *hip_stream, qsv_ctx **out);
qsv_status qsv_destroy(qsv_ctx *ctx);
/* Change the stream later calls are queued on.  The context's scratch
 * buffers are shared by all its calls, so the new stream is made to wait for
 * the work already queued on the old one (an event, no host wait); calls on
 * one context are therefore ordered even across streams. */
qsv_status qsv_set_stream(qsv_ctx *ctx, void *hip_stream);

/*
 * Partition circuits (paper Section 4.1-4.3).  For each of n_circuits
 * circuits (gates[circ_offsets[c] .. circ_offsets[c+1]); circ_offsets holds
 * n_circuits + 1 non-decreasing offsets starting at 0): build the contraction graph and critical-path
 * lengths, score every gate by closeness centrality (Eq. 10-13), cut the gate
 * list into partitions of at most k_local local qubits with the greedy
 * frontier sweep and its two locality exemptions (diagonal gates, non-local
 * controls), repeat one level down for the register stages, and lower the
 * result to device tables (uploaded when ctx is non-NULL; ctx == NULL gives a
 * host-only plan usable with the introspection calls only).
 * k_local == 0 chooses k and the tile shape by timing candidates on the
 * device (autotuner, needs ctx; n_qubits above the default tile): k in
 * {8, 10, 12} below the tile size, eight tile shapes (reg_qubits x
 * 2^log_threads: 5 x 256, 4 x 256, 4 x 512, 5 x 512, 4 x 1024, 3 x 256,
 * 3 x 512, 3 x 1024); each
 * candidate's time is
 * an evenly spaced sample of at most 8 of its partition sweeps on a scratch
 * state (2^n x 8 bytes, freed afterwards) scaled to all partitions.  With
 * QSV_PLAN_TUNE_SPECIALISED the samples run as specialised kernels (also
 * with k_local > 0, then tuning the tile shape only).  The choice is cached
 * per device, circuit, flags and k_local.  tile may be NULL (default shape).
 * The gate array is copied; it is not retained.  The plan is freed by
 * qsv_plan_destroy.
 * Batched plans (n_circuits > 1) keep each whole state on chip: 4 <= n <= 14.
 * Qubit counts: up to 35 with a context (a 2^35-amplitude complex64 state
 * is 256 GiB, the largest that fits the MI355X's 288 GB), up to 40 for
 * host-only plans (ctx NULL: e.g. the whole of a multi-GPU run).
 * Errors: QSV_E_ARG (n_qubits < 1 or above those limits, k_local < 0, qubit out of range,
 * q0 == q1, unknown kind, bad offsets, a batched plan with n_qubits > 14),
 * QSV_E_RANGE (param >= 0 on a non-rotation), QSV_E_NOMEM, QSV_E_DEVICE.
 */
qsv_status qsv_partition(qsv_ctx *ctx, int32_t n_qubits, const qsv_gate *gates, const int64_t *circ_offsets,
                         int32_t n_circuits, int32_t k_local, uint32_t flags, const qsv_tile_config *tile,
                         qsv_plan **out);
qsv_status qsv_plan_destroy(qsv_plan *plan);
qsv_status qsv_plan_get_info(const qsv_plan *plan, qsv_plan_info *out);

/*
 * Specialise a plan's partition sweeps (paper Section 4.3, Step D: the
 * computation of each partition is generated as code).  For every partition
 * a kernel is generated with the partition's tile qubits, register stages,
 * lowered ops and constant gate matrices as compile-time constants. The
 * kernels are compiled for gfx950 with hipRTC in up to 16 helper processes
 * at once and loaded on the context's device.  Afterwards qsv_apply on this plan
 * launches them instead of the table-driven sweep kernel.  The ops, their
 * order and their arithmetic are the same; only the compiler's choice of
 * fused multiply-adds may differ in the last bits.  Matrices of
 * parameterised rotations are still formed from theta at every qsv_apply.
 * Plans made with QSV_PLAN_GRAD whose tiles take at most 12 qubits (psi and
 * lambda tiles together in 64 KiB of LDS) also get one specialised reverse
 * kernel per partition, which qsv_adjoint_grad then launches; other plans
 * keep the table-driven reverse walk.  The forward it starts from (qsv_apply
 * with checkpoints) uses the specialised sweeps.
 * Batched plans (several circuits): one program, holding a version of the
 * persistent batched kernel with the register stages of every circuit
 * structure compiled in (circuits with identical gate records share one;
 * the kernel switches on a circuit's structure).  qsv_apply on the plan then
 * launches it; qsv_adjoint_grad keeps the table-driven reverse walk, from the
 * given final states or (psi_final NULL) from those of a specialised forward
 * launch into a scratch batch of states.  Its compile grows with the total op
 * count of the structures (about two minutes for 13 ansatz structures of 4-16
 * layers on 14 qubits): qsv_plan_specialise_async overlaps it with other work.
 * ctx NULL: generate and compile only, load nothing (a check that needs no
 * GPU); the plan is unchanged.  The compile runs in the helper executable
 * qsv_rtc next to this library.  Environment: QSV_KERNEL_CACHE=<dir> keeps
 * every compiled program in <dir>, keyed by a hash of the program text, the
 * device headers and the compile options, and reuses it; with
 * QSV_KERNEL_CACHE_ONLY=1 as well, a program missing from the cache is an
 * error (QSV_E_DEVICE) and no compiler process is started.  A plan that is
 * already specialised is left as it is.  seconds_out (may be NULL) receives the host time taken
 * (after a background compile: the compile's own duration).
 * Errors: QSV_E_ARG (plan null), QSV_E_UNSUPPORTED (a single-circuit plan
 * with tiles above 13 qubits, i.e. beyond 64 KiB of LDS), QSV_E_STATE
 * (plan without device tables on the context's device), QSV_E_DEVICE (the
 * compile or the load failed: qsv_last_error() holds the compiler log).
 */
qsv_status qsv_plan_specialise(qsv_ctx *ctx, qsv_plan *plan, double *seconds_out);
/*
 * qsv_plan_specialise without waiting for the compile (for plans applied a
 * few times only, where the compile would cost more than it saves): the
 * programs are generated and compiled on a host thread of the library's own,
 * a few partitions per program and the last partitions first (an apply that
 * runs meanwhile reaches them last), and the call returns at once.  Before every sweep, qsv_apply (and qsv_adjoint_grad before its
 * walk) loads the programs that have finished, on the calling thread; each
 * partition launches its specialised kernel once its program is loaded and
 * the table-driven kernel until then.
 * While a compile is pending, qsv_apply keeps at most two sweeps queued ahead
 * of the GPU so that later sweeps can switch.  The results are those of
 * either kernel kind (equal up to the compiler's choice of fused
 * multiply-adds).  qsv_plan_specialise on the plan waits for the compile
 * (QSV_E_DEVICE if it failed; the plan then stays table-driven), and
 * qsv_plan_destroy waits for it and discards it.  The plan must not be used
 * from two threads at once.  A plan already specialised, or with a compile
 * pending, is left as it is.  A batched plan compiles its one program this
 * way; its launches stay table-driven until the program is loaded.
 * Errors: QSV_E_ARG (null), QSV_E_UNSUPPORTED and QSV_E_STATE as for
 * qsv_plan_specialise.
 */
qsv_status qsv_plan_specialise_async(qsv_ctx *ctx, qsv_plan *plan);
/* Number of theta entries of circuit c and its offset in the packed theta array. */
qsv_status qsv_plan_params(const qsv_plan *plan, int32_t circuit, int64_t *offset, int64_t *count);
/*
 * Introspection of partition p of circuit c (Section 4.3 partition tree):
 * local_mask = its local qubit set S (|S| = min(k, n)), gates = its gate
 * indices in execution order (at most cap written; *n_gates = the count).
 * level 0 = the partition level, level 1 = the register stages of all
 * partitions of circuit c in order (local_mask = the stage's register qubits).
 * Distributed plans: level -1 = the distributed partitions (local_mask = the
 * n - n_global logical qubits local to every rank); at levels 0 and 1 the
 * masks are physical bit positions and a remap SWAP's gate index is -1.
 */
/*
 * Distributed level (Section 4.2 with the memory of one rank as the local
 * size, Section 4.3's data reshaping between partitions), emulated on one
 * GPU.  2^n_global ranks each own the 2^(n - n_global) amplitudes whose
 * n_global highest bit positions equal the rank.  The greedy of
 * qsv_partition cuts the circuit (gates[0..n_gates), one circuit) into
 * distributed partitions of at most n - n_global local qubits; the local set
 * is padded with qubits that are already local.  Each distributed partition
 * runs with its local qubits at the low positions (tiles of k local qubits as
 * in qsv_partition, never spanning ranks).  Between partitions every qubit
 * that becomes local trades positions with one that stops being local: one
 * SWAP of a low and a high position, the exchange between the ranks that
 * differ in that high bit.  On one GPU these SWAPs run as sweeps of the same
 * kernels; a final set of SWAPs restores the logical order, so qsv_apply,
 * qsv_expect and qsv_adjoint_grad see the state in logical order.
 * k_local == 0 gives the default k; tile as in qsv_partition.  n_qubits
 * from 2 up to 35 with a context, up to 40 for host-only plans (ctx NULL).
 * Errors: QSV_E_ARG (n_qubits out of range, n_global < 1, fewer than tile-size qubits left local,
 * invalid gates, k_local not below the tile size), QSV_E_RANGE,
 * QSV_E_UNSUPPORTED (gradient plans with tiles over 13 qubits), QSV_E_NOMEM,
 * QSV_E_DEVICE.
 */
qsv_status qsv_partition_distributed(qsv_ctx *ctx, int32_t n_qubits, const qsv_gate *gates, int64_t n_gates,
                                     int32_t n_global, int32_t k_local, uint32_t flags, const qsv_tile_config *tile,
                                     qsv_plan **out);
/* Distributed level of a plan: n_global (0 for other plans), the number of
 * distributed partitions, the remap SWAPs that move data between ranks (one
 * low and one high position) and all remap SWAPs (with the final return to
 * logical order). */
qsv_status qsv_plan_distributed_info(const qsv_plan *plan, int32_t *n_global, int64_t *n_dist_partitions,
                                     int64_t *exchange_swaps, int64_t *remap_swaps);
qsv_status qsv_plan_partition(const qsv_plan *plan, int32_t circuit, int32_t level, int64_t p,
                              uint64_t *local_mask, int32_t *gates, int64_t cap, int64_t *n_gates);

/*
 * Apply the planned circuits in place: psi_b <- C_b(theta_b) psi_b on
 * complex64[n_circuits][2^n] (the caller initialises psi, e.g. to |0..0>).
 * Batched plans (n_circuits > 1) always start from |0..0> and write the final
 * states into psi (one persistent launch).
 * theta_dev: float64 device array of qsv_plan_info.n_params entries (may be
 * NULL when the plan has none); rotation matrices are formed on the device
 * (cos/sin in float64, rounded to float32).  When ckpt_dev is non-NULL
 * (single-circuit plans) the state after every partition but the last is also
 * written to ckpt_dev + p * 2^n amplitudes (qsv_plan_info.ckpt_bytes) for
 * qsv_adjoint_grad.
 * Errors: QSV_E_ARG (null psi, theta missing), QSV_E_DEVICE.
 */
qsv_status qsv_apply(qsv_ctx *ctx, const qsv_plan *plan, const double *theta_dev, void *psi_dev,
                     void *ckpt_dev);

/*
 * Expectation values out_b = sum_t coeff_t <psi_b|P_t|psi_b> for b < batch,
 * computed with float64 accumulation into out_dev (float64[batch], device).
 * H = one term with empty masks and coeff 1 gives the squared norm.
 * The context keeps the grouped tables of the last sum on the device: a call
 * with the same terms (byte for byte) and n_qubits skips grouping and upload.
 * Errors: QSV_E_ARG (n_qubits out of range, masks beyond n_qubits, nulls).
 */
qsv_status qsv_expect(qsv_ctx *ctx, const qsv_pauli_term *H, int32_t n_terms, int32_t n_qubits, int64_t batch,
                      const void *psi_dev, double *out_dev);

/*
 * qsv_expect for callers that cannot allocate memory: code recorded under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, same kernels and the same results (bit for bit) as
 * qsv_expect, but the call allocates nothing, on the device or pinned: its
 * scratch (the grouped Pauli terms, then the per-block float64 partial sums)
 * is one static device array of 4 MiB per GPU, in the library's own device
 * memory and held until the process ends; qsv_create looks up its address on
 * the context's device.  The terms are staged through a 512 KiB pinned buffer
 * that qsv_create allocates for each context.
 * Limits: at most 4096 terms, and at most 3.5 MiB of partial sums, i.e.
 * 8 x min(1024, 2^(n-12)) x (tile passes, at least 1) x batch bytes, where a
 * pass covers the X/Y masks that fit one 12-qubit tile together with qubits
 * 0-3 (for example n = 28 allows passes x batch <= 448).
 * Sharing: every call on one GPU uses that GPU's one array, from any context
 * or stream.  Calls that overlap on one GPU race (two streams, contexts or
 * threads) and must be ordered by the caller.  The array keeps the last
 * call's contents; each call writes every value it reads before reading it,
 * so nothing needs to start at zero.  Before reusing the staging buffer the
 * call waits (host side) for its previous copy on this context's stream.
 * Errors: those of qsv_expect; QSV_E_RANGE (more than 4096 terms, or partial
 * sums beyond the scratch); QSV_E_STATE (no scratch address on the device).
 */
qsv_status qsv_expect_noalloc(qsv_ctx *ctx, const qsv_pauli_term *H, int32_t n_terms, int32_t n_qubits,
                              int64_t batch, const void *psi_dev, double *out_dev);

/*
 * Adjoint gradient (reverse sweep over the partitions).  For every circuit b:
 * energy_b = <psi_b|H|psi_b> and grad_b[j] = d energy_b / d theta_b[j]
 * (parameters used by several rotations receive the sum of their terms).
 * Single-circuit plans: psi_final_dev is the state qsv_apply produced and
 * ckpt_dev the checkpoints it wrote; the plan must carry QSV_PLAN_GRAD.
 * Batched plans (n_circuits > 1): energy and adjoint of every circuit run in
 * one persistent launch (longest circuits first); ckpt_dev is ignored.
 * psi_final_dev is either the final states qsv_apply wrote for this plan and
 * theta (complex64[n_circuits][2^n], read only) or NULL, in which case the
 * same launch first runs each circuit forward from |0..0>.
 * grad_dev: float64[n_params], energy_dev: float64[n_circuits].
 * Errors: QSV_E_STATE (no QSV_PLAN_GRAD or missing checkpoints), QSV_E_ARG.
 */
qsv_status qsv_adjoint_grad(qsv_ctx *ctx, const qsv_plan *plan, const qsv_pauli_term *H, int32_t n_terms,
                            const double *theta_dev, const void *psi_final_dev, const void *ckpt_dev,
                            double *energy_dev, double *grad_dev);

/* Candidates timed by the last autotuning run in this process (k_local == 0,
 * or QSV_PLAN_TUNE_SPECIALISED, on a context): writes up to cap records of 4 int32 (k, reg_qubits,
 * log_threads, estimated microseconds for the whole circuit) and returns the
 * number of candidates. */
int32_t qsv_last_autotune(int32_t *out, int32_t cap);

/* Time-stamped launch counters of the last call on ctx (for benchmarks):
 * average duration in ms of the sweep kernels of the last qsv_apply, measured
 * with HIP events on the context stream when timing is enabled. */
qsv_status qsv_set_timing(qsv_ctx *ctx, int32_t enable);
qsv_status qsv_last_sweep_ms(qsv_ctx *ctx, double *total_ms, int64_t *n_launches);
/* The duration in ms of each sweep launch of the last qsv_apply on ctx (in
 * partition order; at most cap written to ms_out, host memory), measured with
 * the same HIP events when timing is enabled; *n_launches = the number of
 * launches (0 when timing was off).  Waits for the last launch to finish. */
qsv_status qsv_last_sweep_times(qsv_ctx *ctx, float *ms_out, int64_t cap, int64_t *n_launches);
/* Load balance of the last batched launch on ctx made with timing enabled
 * (batched plans: one persistent launch, workgroups taking circuits from a
 * queue): for each of its *n_workgroups workgroups, the device's real-time
 * clock when it started and when it exited (2 values per workgroup, at most
 * cap written to ticks_out, host memory); *ticks_per_s (may be NULL) receives
 * the clock's rate.  Waits for the context's stream.  *n_workgroups is 0 when
 * the last batched launch ran without timing. */
qsv_status qsv_last_batch_clock(qsv_ctx *ctx, uint64_t *ticks_out, int64_t cap, int64_t *n_workgroups,
                                double *ticks_per_s);

#ifdef __cplusplus
}
#endif

#endif /* QSV_PUBLIC_API_H_ */
