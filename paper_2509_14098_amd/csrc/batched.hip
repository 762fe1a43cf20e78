// Batched persistent kernel, table-driven: the body of batched.cuh with a walk
// that reads the plan's stage and op tables at run time (the specialised
// programs of qsv_plan_specialise walk a circuit structure compiled in).
#include <hip/hip_runtime.h>

#include "batched.cuh"
#include "kernels.h"

namespace qsv {

template <int R, int LW>
__global__ __launch_bounds__(1 << LW) void batched_kernel(
    const DevPart *__restrict__ parts, const DevStage *__restrict__ stages, const DevOp *__restrict__ ops,
    const float *__restrict__ pool, const int32_t *__restrict__ order, const int32_t *__restrict__ circ_part,
    const int64_t *__restrict__ circ_theta, const int64_t *__restrict__ circ_npar,
    const int32_t *__restrict__ param_off, const int32_t *__restrict__ param_slots,
    const int32_t *__restrict__ circ_pool_delta, const int32_t *__restrict__ circ_slot_delta,
    const DevGroup *__restrict__ groups, const DevTerm *__restrict__ terms, BatchArgs A)
{
    batched_body<R, LW, TableWalk<R, LW>>(parts, stages, ops, pool, order, circ_part, circ_theta, circ_npar, param_off,
                                          param_slots, circ_pool_delta, circ_slot_delta, groups, terms, A);
}

__global__ void reset_counter_kernel(int *q)
{
    if (threadIdx.x == 0) *q = 0;
}

constexpr int BATCH_R = 4, BATCH_LW = 10;

template <int R, int LW>
static void set_lds_attr()
{
    static bool done = false;
    if (!done) {
        (void)hipFuncSetAttribute((const void *)batched_kernel<R, LW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipGetLastError();
        done = true;
    }
}

hipError_t launch_batched(const Plan &plan, const DevGroup *groups, int n_groups, const DevTerm *terms,
                          const double *theta, float2 *psi_out, const float2 *psi_in, double *energy, double *grad,
                          double *gpart, int *queue, bool adjoint, int grid, uint64_t *wg_clock, hipStream_t s)
{
    if (plan.R != BATCH_R || plan.LW != BATCH_LW) return hipErrorInvalidValue;
    // the specialised forward applies folded RZ diagonals as their members' own
    // rotations: their 2^R-entry tables are not needed there
    hipError_t e = launch_materialize(plan, theta, s, !(plan.spec_batch_fn && !adjoint));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, queue);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchArgs A;
    A.n_groups = n_groups;
    A.n_circuits = plan.n_circuits;
    A.n = plan.n;
    A.psi_out = psi_out;
    A.psi_in = adjoint ? psi_in : nullptr;
    A.energy = energy;
    A.grad = grad;
    A.gpart = gpart;
    A.queue = queue;
    A.adjoint = adjoint ? 1 : 0;
    A.wg_clock = wg_clock;
    const size_t lds = (size_t)8 << plan.t;
    if (plan.spec_batch_fn && !adjoint) {  // the kernel specialised for the plan's circuit structures
        const DevPart *parts = plan.d_parts;
        const DevStage *stages = plan.d_stages;
        const DevOp *ops = plan.d_ops;
        const float *pool = plan.d_pool;
        const int32_t *order = plan.d_batch_order, *cpart = plan.d_circ_part;
        const int64_t *ctheta = plan.d_circ_theta, *cnpar = plan.d_circ_npar;
        const int32_t *poff = plan.d_param_off, *pslots = plan.d_param_slots;
        const int32_t *pdelta = plan.d_circ_pool_delta, *sdelta = plan.d_circ_slot_delta;
        void *args[] = {&parts, &stages, &ops, &pool, &order, &cpart, &ctheta, &cnpar, &poff, &pslots,
                        &pdelta, &sdelta, &groups, &terms, &A};
        return hipModuleLaunchKernel((hipFunction_t)plan.spec_batch_fn, (uint32_t)grid, 1, 1, 1u << BATCH_LW, 1, 1,
                                     (uint32_t)lds, s, args, nullptr);
    }
    set_lds_attr<BATCH_R, BATCH_LW>();
    hipLaunchKernelGGL((batched_kernel<BATCH_R, BATCH_LW>), dim3(grid), dim3(1 << BATCH_LW), lds, s, plan.d_parts,
                       plan.d_stages, plan.d_ops, plan.d_pool, plan.d_batch_order, plan.d_circ_part,
                       plan.d_circ_theta, plan.d_circ_npar, plan.d_param_off, plan.d_param_slots,
                       plan.d_circ_pool_delta, plan.d_circ_slot_delta, groups, terms, A);
    return hipGetLastError();
}

int batched_waves() { return (1 << BATCH_LW) / 64; }

}  // namespace qsv
