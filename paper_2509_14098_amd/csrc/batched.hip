// Batched persistent kernel: many small circuits (n <= 14) with uneven depths,
// each run entirely on chip by one workgroup.
//
// The grid holds one workgroup per compute unit.  A workgroup takes the next
// circuit from a device queue (circuits ordered by decreasing work, so the
// longest start first) until the queue is empty; every workgroup reaches that
// exit.  Per circuit:
//   forward  — |0..0> in LDS, the register stages of the circuit (one
//              partition covers the whole state), final state optionally
//              written out;
//   energy   — lambda = H psi in the last stage's register layout, reading the
//              partner amplitudes of each Pauli group from LDS; <H> reduced in
//              float64 in a fixed order;
//   adjoint  — stages walked backwards with psi and lambda both in registers,
//              remapped between stage layouts through LDS; for every
//              parameterised rotation Im <lambda|P|psi> is summed per wave
//              (float64) before U^dagger is applied to both states; the
//              circuit's gradient entries are then reduced in a fixed order.
#include <hip/hip_runtime.h>

#include "gates.cuh"
#include "kernels.h"

namespace qsv {

// The read-only tables (plan and Hamiltonian) are separate restrict kernel
// arguments: the compiler then knows the kernel's stores cannot change them
// and fetches ops and matrices with scalar loads.
struct BatchArgs {
    int n_groups;
    int n_circuits;
    int n;
    float2 *psi_out;            // forward only: final states (may be null)
    const float2 *psi_in;       // adjoint only: final states of the forward (null: recompute them)
    double *energy;             // [n_circuits] (adjoint only)
    double *grad;               // [n_params]   (adjoint only)
    double *gpart;              // [n_slots][waves] scratch
    int *queue;
    int adjoint;
    uint64_t *wg_clock;         // null, or per workgroup the real-time clock at its start and at its exit
};

// Registers in the layout (toff, roff) -> LDS -> registers in the layout (toff2,
// roff2); offsets are already swizzled.
template <int R>
__device__ __forceinline__ void remap(float2 (&v)[1 << R], float2 *lds, bool active, uint32_t toff,
                                      const uint32_t (&roff)[1 << R], uint32_t toff2, const uint32_t (&roff2)[1 << R])
{
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) lds_ref(lds, toff ^ roff[i]) = v[i];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) v[i] = lds_ref(lds, toff2 ^ roff2[i]);
    }
}

template <int R, int LW>
__global__ __launch_bounds__(1 << LW) void batched_kernel(
    const DevPart *__restrict__ parts, const DevStage *__restrict__ stages, const DevOp *__restrict__ ops,
    const float *__restrict__ pool, const int32_t *__restrict__ order, const int32_t *__restrict__ circ_part,
    const int64_t *__restrict__ circ_theta, const int64_t *__restrict__ circ_npar,
    const int32_t *__restrict__ param_off, const int32_t *__restrict__ param_slots,
    const int32_t *__restrict__ circ_pool_delta, const int32_t *__restrict__ circ_slot_delta,
    const DevGroup *__restrict__ groups, const DevTerm *__restrict__ terms, BatchArgs A)
{
    constexpr int NA = 1 << R, WAVES = (1 << LW) / 64;
    extern __shared__ float2 lds[];
    __shared__ int s_item;
    __shared__ double s_red[WAVES];
    const uint32_t tid = threadIdx.x;
    const int wave = tid >> 6;
    if (A.wg_clock && tid == 0) A.wg_clock[2 * blockIdx.x] = __builtin_amdgcn_s_memrealtime();
    while (true) {
        if (tid == 0) s_item = atomicAdd(A.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // the same for every thread
        __syncthreads();
        if (item >= A.n_circuits) break;
        const int c = order[item];
        // circuits of the same structure share their tables: this circuit's own
        // matrices and gradient slots sit at a constant offset from the ones the
        // tables name
        const DevPart *__restrict__ P = parts + circ_part[c];
        const float *__restrict__ cpool = pool + circ_pool_delta[c];
        const int32_t slot_delta = circ_slot_delta[c];
        const int t = P->t, w = t - R;
        const bool active = tid < (1u << w);
        const uint32_t dim = 1u << t;
        if (A.psi_in) {  // the forward's final state (positions are the qubits in order)
            const float2 *src = A.psi_in + (uint64_t)c * dim;
            for (uint32_t x = tid; x < dim; x += (1u << LW)) lds[swz(x)] = src[x];
            __syncthreads();
        } else {  // forward from |0..0>
            for (uint32_t x = tid; x < dim; x += (1u << LW)) lds[swz(x)] = float2{x == 0 ? 1.f : 0.f, 0.f};
            __syncthreads();
            run_stages<R, false>(lds, stages, ops, cpool, P->stage_begin, P->stage_end, w, tid, 0);
        }
        if (A.psi_out) {  // the tile is the whole state and its positions are the qubits in order
            float2 *dst = A.psi_out + (uint64_t)c * dim;
            for (uint32_t x = tid; x < dim; x += (1u << LW)) dst[x] = lds[swz(x)];
        }
        if (!A.adjoint) {
            __syncthreads();
            continue;
        }
        // lambda = H psi and the energy, in the last stage's layout
        const int s_last = P->stage_end - 1;
        uint32_t toff, roff[NA];
        stage_offsets<R>(stages + s_last, w, tid, toff, roff);
        float2 a[NA], l[NA];
        double e_part = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            a[i] = float2{0.f, 0.f};
            l[i] = float2{0.f, 0.f};
            if (active) {
                const uint32_t sx = (toff ^ roff[i]) >> 3;  // swizzled slot of amplitude x
                const uint32_t x = swz(sx);          // swz is an involution here: recovers x
                a[i] = lds[sx];
                double lr = 0.0, li = 0.0;
                for (int g = 0; g < A.n_groups; ++g) {
                    const DevGroup G = groups[g];
                    const uint32_t y = x ^ (uint32_t)G.x_mask;
                    const float2 py = lds[swz(y)];
                    double wr = 0.0, wi = 0.0;
                    for (int k = G.term_begin; k < G.term_end; ++k) {
                        const double sg = (__popcll(y & terms[k].z_mask) & 1) ? -1.0 : 1.0;
                        wr += sg * terms[k].cre;
                        wi += sg * terms[k].cim;
                    }
                    lr += wr * py.x - wi * py.y;
                    li += wr * py.y + wi * py.x;
                }
                l[i] = float2{(float)lr, (float)li};
                e_part += (double)a[i].x * lr + (double)a[i].y * li;
            }
        }
        e_part = wave_sum(e_part);
        if ((tid & 63) == 0) s_red[wave] = e_part;
        __syncthreads();
        if (tid == 0) {
            double e = 0.0;
            for (int v = 0; v < WAVES; ++v) e += s_red[v];
            A.energy[c] = e;
        }
        // reverse walk over the stages
        for (int s = s_last; s >= P->stage_begin; --s) {
            if (s != s_last) {  // remap psi, then lambda, from the layout of stage s+1 to that of stage s
                uint32_t toff2, roff2[NA];
                stage_offsets<R>(stages + s, w, tid, toff2, roff2);
                remap<R>(a, lds, active, toff, roff, toff2, roff2);
                remap<R>(l, lds, active, toff, roff, toff2, roff2);
                toff = toff2;
#pragma unroll
                for (int i = 0; i < NA; ++i) roff[i] = roff2[i];
            }
            const DevStage *__restrict__ S = stages + s;
            for (int k = S->op_end - 1; k >= S->op_begin; --k) {
                const DevOp o = ops[k];
                if (o.grad_slot >= 0) {
                    const double v = wave_sum(grad_term<R>(a, l, o, tid, 0));
                    if ((tid & 63) == 0) A.gpart[(int64_t)(o.grad_slot + slot_delta) * WAVES + wave] = v;
                }
                // one array at a time: with 1024 threads a lane has 128 VGPRs, too
                // few to update psi and lambda together without spilling
                apply_op<R, true>(a, o, cpool, tid, 0);
                apply_op<R, true>(l, o, cpool, tid, 0);
            }
        }
        // this circuit's gradient entries: slots in slot order, waves in order
        __threadfence_block();
        __syncthreads();
        const int64_t p0 = circ_theta[c], np = circ_npar[c];
        for (int64_t p = tid; p < np; p += (1 << LW)) {
            double acc = 0.0;
            for (int32_t k = param_off[p0 + p]; k < param_off[p0 + p + 1]; ++k)
                for (int v = 0; v < WAVES; ++v) acc += A.gpart[(int64_t)param_slots[k] * WAVES + v];
            A.grad[p0 + p] = acc;
        }
        __syncthreads();
    }
    if (A.wg_clock && tid == 0) A.wg_clock[2 * blockIdx.x + 1] = __builtin_amdgcn_s_memrealtime();
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
    hipError_t e = launch_materialize(plan, theta, s);
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
    set_lds_attr<BATCH_R, BATCH_LW>();
    hipLaunchKernelGGL((batched_kernel<BATCH_R, BATCH_LW>), dim3(grid), dim3(1 << BATCH_LW), lds, s, plan.d_parts,
                       plan.d_stages, plan.d_ops, plan.d_pool, plan.d_batch_order, plan.d_circ_part,
                       plan.d_circ_theta, plan.d_circ_npar, plan.d_param_off, plan.d_param_slots,
                       plan.d_circ_pool_delta, plan.d_circ_slot_delta, groups, terms, A);
    return hipGetLastError();
}

int batched_waves() { return (1 << BATCH_LW) / 64; }

}  // namespace qsv
