// Kernel launchers (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace qsv {

bool kernel_shape_supported(int R, int LW);
hipError_t launch_sweep(const Plan &plan, int R, int LW, int pidx, float2 *psi, float2 *ckpt, hipStream_t s);
// Rotation matrices (and, with diags, the register diagonals folded from
// parameterised RZ rotations) formed from theta in the plan's pool.
hipError_t launch_materialize(const Plan &plan, const double *theta, hipStream_t s, bool diags = true);

// expect.hip
constexpr int EXPECT_TILE_QUBITS = 12;   // tiles of 4096 amplitudes, 32 KiB of LDS
constexpr int EXPECT_LOG_THREADS = 9;   // 512 threads per workgroup
constexpr int EXPECT_THREADS = 1 << EXPECT_LOG_THREADS;
constexpr int EXPECT_PAIRS = (1 << EXPECT_TILE_QUBITS) / (2 * EXPECT_THREADS);  // amplitude pairs per thread: 4
constexpr int EXPECT_MAX_BLOCKS = 1024; // workgroups per (pass, batch entry)
constexpr int EXPECT_MIN_BLOCKS = 512;  // passes are split by groups until they fill this many workgroups
constexpr int EXPECT_LDS_GROUPS = 128;  // a pass's group and term tables are copied to LDS up to these sizes
constexpr int EXPECT_LDS_TERMS = 256;
constexpr int EXPECT_CACHED_QUBITS = 24;  // states up to 128 MiB are read through the caches (several passes)
// Workgroups per (pass, batch entry): partial sums of launch_expect are
// n_passes x expect_blocks(n) x batch doubles.
int expect_blocks(int n);
// Cuts groups (sorted by increasing X mask) into passes (at most n_groups),
// sets each group's xt and each of its terms' zt; returns the number of
// passes.  Allocates nothing.
int plan_expect_passes(int n, DevGroup *groups, int n_groups, DevTerm *terms, DevPass *passes);
hipError_t launch_expect(const DevPass *passes, int n_passes, const DevGroup *groups, const DevTerm *terms, int n,
                         int64_t batch, const float2 *psi, double *partials, double *out, hipStream_t s);
// The fixed scratch of qsv_expect_noalloc (one per device): the grouped
// Pauli terms, then the per-block partial sums.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(4) << 20;
constexpr size_t NOALLOC_TERMS_BYTES = size_t(512) << 10;
constexpr int NOALLOC_MAX_TERMS = 4096;   // 4096 x (DevTerm + DevGroup + DevPass) fit NOALLOC_TERMS_BYTES
constexpr int NOALLOC_MAX_DEVICES = 64;
static_assert(NOALLOC_MAX_TERMS * (sizeof(DevTerm) + sizeof(DevGroup) + sizeof(DevPass)) + 32 <= NOALLOC_TERMS_BYTES,
              "terms region");
// Looks up the array's address on `device`, which must be the current device;
// once per device (later calls return at once).
hipError_t noalloc_scratch_init(int device);
// The address found by noalloc_scratch_init, or null before it ran.
void *noalloc_scratch(int device);
// Blocks launch_apply_h uses for 2^n amplitudes and a cap (one partial each).
int apply_h_blocks(int n, int cap);
hipError_t launch_apply_h(const DevGroup *groups, int n_groups, const DevTerm *terms, int n, const float2 *psi,
                          float2 *lam, double *partials, int n_blocks, double *energy, hipStream_t s);

// adjoint.hip
hipError_t launch_reverse(const Plan &plan, int R, int LW, int pidx, const float2 *psi_ckpt, float2 *lam,
                          double *gpart, int64_t n_tiles_stride, hipStream_t s);
hipError_t launch_grad_reduce(const Plan &plan, const double *gpart, int64_t n_slots, int64_t stride,
                              double *slot_sum, double *grad, hipStream_t s);

// batched.hip
hipError_t launch_batched(const Plan &plan, const DevGroup *groups, int n_groups, const DevTerm *terms,
                          const double *theta, float2 *psi_out, const float2 *psi_in, double *energy, double *grad,
                          double *gpart, int *queue, bool adjoint, int grid, uint64_t *wg_clock, hipStream_t s);
int batched_waves();

}  // namespace qsv
