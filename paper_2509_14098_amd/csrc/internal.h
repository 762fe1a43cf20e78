// Host-side structures shared by the planner, the C interface and the kernel
// launchers.  Not part of the public interface.
#pragma once
#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "plan.h"

namespace qsv {

// Classification of one gate, from the exact zeros of its float64 matrix
// (fixed gates) or from the structure of its kind (parameterised rotations).
struct GateMeta {
    int nq = 1;
    int q[2] = {-1, -1};
    uint64_t qmask = 0;   // all qubits of the gate
    uint64_t req = 0;     // qubits that must be local (Section 4.2 exemptions)
    OpKind op = OP_U1;    // register-level kernel path
    int ctrl = -1, tgt = -1;  // for OP_CX / OP_CU
    GenKind gen = GEN_NONE;
    bool param = false;
    double m[32] = {0};   // float64 matrix (fixed gates), (re, im) row-major
    double flops = 0;     // algorithmic flops per amplitude
};

// A partition at some level: local qubit set and gate indices in order.
struct Part {
    uint64_t S = 0;
    std::vector<int> gates;
};

struct CircuitPlan {
    int64_t g0 = 0, g1 = 0;          // gate range in the plan's gate array
    int64_t theta_off = 0, n_params = 0;
    std::vector<Part> parts;          // level 1 (tile / LDS)
    std::vector<std::vector<Part>> stages;  // level 2 (registers), per partition
    int32_t part_begin = 0;           // index of its first DevPart
    int32_t shares = -1;              // batched: the circuit whose tables this one reuses, or -1
};

// A run of the plan's gate list partitioned on its own at the tile level:
// the gates of one distributed partition (qubits relabelled to physical bit
// positions, tiles restricted to the rank-local positions in allowed) or the
// SWAPs of one remap between distributed partitions (any positions).
struct Segment {
    int64_t g0 = 0, g1 = 0;
    uint64_t allowed = ~0ull;
    bool remap = false;
};

struct ParamGate {                    // a rotation whose matrix is formed from theta on the device
    int32_t mat;                      // pool offset
    int32_t kind;
    int32_t theta_index;              // absolute index into the packed theta array
    int32_t pad;
};

// A register diagonal formed on the device from the angles of the RZ rotations
// it folds (one per member register slot, slots in increasing order): entry u
// is exp(i/2 sum_m (2 u_{slot m} - 1) theta_m).  Its op is an OP_DREG whose
// field a holds the member slots' mask and whose gradient slots are
// grad_slot + m for member m.
struct ParamDiag {
    int32_t mat;                      // pool offset of its 2^R complex entries
    int32_t n;                        // members
    int32_t slot[MAX_R];
    int32_t theta[MAX_R];             // absolute theta index of each member
    int32_t gmat[MAX_R];              // pool offset of each member's own RZ matrix
};

struct Plan {
    int n = 0, n_circuits = 0, k = 0, t = 0, R = 0, LW = 0;
    uint32_t flags = 0;
    std::vector<qsv_gate> gates;
    std::vector<GateMeta> meta;
    std::vector<CircuitPlan> circ;
    int64_t n_params = 0;
    double plan_seconds = 0, flops = 0, bytes = 0;

    // lowered tables
    std::vector<DevOp> ops;
    std::vector<DevStage> stages;
    std::vector<DevPart> parts;
    std::vector<float> pool;
    std::vector<ParamGate> pgates;
    std::vector<ParamDiag> pdiags;    // register diagonals folded from parameterised RZ rotations
    std::vector<int32_t> grad_param;  // grad slot -> absolute theta index
    std::vector<int32_t> param_off, param_slots;  // theta index -> its grad slots (CSR, slot order)
    // batched plans: per-circuit stage ranges (single tile per circuit)
    std::vector<int32_t> batch_order; // circuits sorted by decreasing op count
    std::vector<int32_t> circ_pool_delta;  // batched: pool offset of a circuit against the tables it uses
    std::vector<int32_t> circ_slot_delta;  // batched: gradient slot offset likewise
    // distributed plans (n_global > 0): the circuit's level above the tile
    int n_global = 0;
    std::vector<Part> dist_parts;     // distributed partitions: local set (logical qubits) and logical gates
    std::vector<Segment> segments;    // how the physical gate list is cut at the tile level
    std::vector<int64_t> phys_logical;  // physical gate -> logical gate index, -1 for a remap SWAP
    int64_t remap_exchange_swaps = 0; // remap SWAPs between a rank-local and a global position
    int64_t remap_swaps = 0;          // all remap SWAPs (including the final return to logical order)
    // specialised sweeps (qsv_plan_specialise): per partition a hipFunction_t, null for none
    std::vector<void *> spec_fn;
    std::vector<void *> spec_rev_fn;  // the adjoint walk's kernels (gradient plans with tiles of 12 qubits or fewer)
    std::vector<void *> spec_modules; // hipModule_t, unloaded with the plan
    void *spec_batch_fn = nullptr;    // batched plans: the specialised qsv_bspec (hipFunction_t), or null
    bool specialised = false;
    double specialise_seconds = 0;
    // qsv_plan_specialise_async: the compile running in the background (null
    // when none is pending); its kernels are loaded by the next call on the plan
    // that finds it finished
    std::shared_ptr<struct AsyncSpecialise> async_spec;
    std::string specialise_error;     // the error of a failed background compile

    // device copies (null for host-only plans)
    int device = -1;
    DevOp *d_ops = nullptr;
    DevStage *d_stages = nullptr;
    DevPart *d_parts = nullptr;
    float *d_pool = nullptr;
    ParamGate *d_pgates = nullptr;
    ParamDiag *d_pdiags = nullptr;
    int32_t *d_grad_param = nullptr;
    int32_t *d_param_off = nullptr;
    int32_t *d_param_slots = nullptr;
    int32_t *d_batch_order = nullptr;  // batched: queue position -> circuit
    int32_t *d_circ_part = nullptr;    // batched: circuit -> its DevPart
    int64_t *d_circ_theta = nullptr;   // batched: theta offset per circuit
    int64_t *d_circ_npar = nullptr;    // batched: parameter count per circuit
    int32_t *d_circ_pool_delta = nullptr;  // batched: per circuit
    int32_t *d_circ_slot_delta = nullptr;  // batched: per circuit
};

// planner.cpp
std::string validate_gate(const qsv_gate &g, int n, int64_t n_params_hint);
GateMeta classify(const qsv_gate &g);
std::vector<Part> greedy_partition(int n, const std::vector<GateMeta> &meta, const std::vector<int> &sub, int k,
                                   uint64_t allowed);
void build_plan(Plan &plan);
// Distributed level: sets plan.gates to the physical gate list of the logical
// circuit gates[0..G) for 2^n_global ranks (plan.n set), and the segments,
// distributed partitions and gate map.
void distribute(Plan &plan, const qsv_gate *gates, int64_t G, int n_global);

// specialise.cpp (program text) and rtc_driver.cpp (compilation): generated
// sweep kernels, one per partition, compiled with hipRTC.  Partitions [p0, p1)
// share one program and code object.
struct SpecChunk {
    int p0 = 0, p1 = 0;
    std::vector<char> code;
};
std::string specialise_source(const Plan &plan, int p0, int p1, bool with_reverse);
// The program of a batched plan's specialised kernel qsv_bspec (one program:
// the persistent kernel switches between the plan's circuit structures).
std::string specialise_batched_source(const Plan &plan);
// Compiles it (one helper process, through the code-object cache); "" or the error.
std::string specialise_batched_compile(const Plan &plan, std::vector<char> &code);
// Whether the adjoint walk is specialised too: gradient plans whose psi and
// lambda tiles fit 64 KiB of LDS together.
bool specialise_reverse(const Plan &plan);
// Compiles the partitions of a single-circuit plan (every one, forward and,
// where specialise_reverse holds, reverse kernels; or only the forward kernels
// of the listed partitions, one program each) in up to max_procs compiler
// processes; returns "" or the error (with the compiler log).
// Incremental use (qsv_plan_specialise_async): with chunk_partitions > 0 the
// partitions are cut into programs of that many partitions, compiled last
// partitions first; on_sized(n) is called once chunks holds all n programs
// (before any compile), and on_chunk(c), on the calling thread, as soon as
// program c's code object is in chunks[c].
std::string specialise_compile(const Plan &plan, std::vector<SpecChunk> &chunks, int max_procs,
                               const std::vector<int> *subset = nullptr, int chunk_partitions = 0,
                               const std::function<void(size_t)> &on_chunk = nullptr,
                               const std::function<void(size_t)> &on_sized = nullptr);

}  // namespace qsv
