// Adjoint (reverse-sweep) gradient over the partitions.
//
// For partition p, walked from the last to the first: a workgroup loads the
// tile of the checkpointed state after p (psi) and of lambda, then walks the
// partition's register stages and gates backwards.  For a parameterised
// rotation exp(-i a P / 2) it first adds Im <lambda|P|psi> over its amplitudes
// (both states taken just after the gate; float64 products and sums), then
// applies U^dagger to psi and to lambda.  lambda goes back to HBM, psi is
// dropped (the next partition reloads its own checkpoint).  Per-wave partial
// sums are written per (gate, tile, wave) and reduced in a fixed order.
#include <hip/hip_runtime.h>

#include "gates.cuh"
#include "kernels.h"
#include "tile.cuh"

namespace qsv {

template <int R, int LW>
__global__ __launch_bounds__(1 << LW) void reverse_kernel(const float2 *__restrict__ psi_src, float2 *__restrict__ lam,
                                                            const DevPart *__restrict__ parts, int pidx,
                                                            const DevStage *__restrict__ stages,
                                                            const DevOp *__restrict__ ops,
                                                            const float *__restrict__ pool,
                                                            double *__restrict__ gpart, int64_t slot_stride)
{
    constexpr int NA = 1 << R;
    extern __shared__ float2 lds[];
    const DevPart *__restrict__ P = parts + pidx;
    const uint32_t tid = threadIdx.x;
    const int t = P->t;
    float2 *lds_psi = lds, *lds_lam = lds + (1u << t);
    const uint64_t tile = xcd_tile(blockIdx.x, gridDim.x, P);
    uint64_t base = 0;
    for (int b = 0; b < P->n_glb; ++b)
        if ((tile >> b) & 1ull) base |= 1ull << P->gq[b];
    load_pairs<LW>(psi_src, lds_psi, P, base, tid);
    load_pairs<LW>(lam, lds_lam, P, base, tid);
    __syncthreads();
    const int w = t - R;
    const bool active = tid < (1u << w);
    const int waves = (1 << LW) >= 64 ? (1 << LW) / 64 : 1;
    const int64_t part_index = (int64_t)blockIdx.x * waves + (tid >> 6);
    for (int s = P->stage_end - 1; s >= P->stage_begin; --s) {
        const DevStage *__restrict__ S = stages + s;
        uint32_t toff, roff[NA];
        stage_offsets<R>(S, w, tid, toff, roff);
        float2 a[NA], l[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            a[i] = active ? lds_ref(lds_psi, toff ^ roff[i]) : float2{0.f, 0.f};
            l[i] = active ? lds_ref(lds_lam, toff ^ roff[i]) : float2{0.f, 0.f};
        }
        for (int k = S->op_end - 1; k >= S->op_begin; --k) {
            const DevOp o = ops[k];
            if (o.grad_slot >= 0)
                grad_partials<R>(a, l, o, tid, base, [&](int32_t slot, double v) __attribute__((always_inline)) {
                    if ((tid & 63) == 0) gpart[(int64_t)slot * slot_stride + part_index] = v;
                });
            apply_op_dag2<R>(a, l, o, pool, tid, base);
        }
        if (active) {
            asm volatile("" : "+v"(toff));  // recompute the write-back addresses instead of keeping 2^R live
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                lds_ref(lds_psi, toff ^ roff[i]) = a[i];
                lds_ref(lds_lam, toff ^ roff[i]) = l[i];
            }
        }
        __syncthreads();
    }
    store_pairs<LW>(lam, lds_lam, P, base, tid);
}

// slot_sum[s] = sum over (tile, wave) of gpart[s * stride + i], fixed order
__global__ __launch_bounds__(256) void slot_sum_kernel(const double *__restrict__ gpart, int64_t stride,
                                                        double *__restrict__ slot_sum)
{
    __shared__ double sh[256];
    const int64_t s = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < stride; i += 256) acc += gpart[s * stride + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) slot_sum[s] = sh[0];
}

// grad[p] = sum of its slots in slot order
__global__ void param_sum_kernel(const int32_t *__restrict__ off, const int32_t *__restrict__ slots,
                                 const double *__restrict__ slot_sum, int64_t n_params, double *__restrict__ grad)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    double acc = 0.0;
    for (int32_t k = off[p]; k < off[p + 1]; ++k) acc += slot_sum[slots[k]];
    grad[p] = acc;
}

template <int R, int LW>
static hipError_t launch_reverse_t(const Plan &plan, int pidx, const float2 *psi, float2 *lam, double *gpart,
                                   int64_t stride, hipStream_t s)
{
    const DevPart &P = plan.parts[pidx];
    const size_t lds = (size_t)16 << P.t;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)reverse_kernel<R, LW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipGetLastError();
        attr = true;
    }
    if (!plan.spec_rev_fn.empty() && plan.spec_rev_fn[pidx]) {  // the partition's specialised walk
        const float *pool = plan.d_pool;
        void *args[] = {&psi, &lam, &pool, &gpart, &stride};
        return hipModuleLaunchKernel((hipFunction_t)plan.spec_rev_fn[pidx], (uint32_t)(1ull << P.n_glb), 1, 1,
                                     1u << LW, 1, 1, (uint32_t)lds, s, args, nullptr);
    }
    hipLaunchKernelGGL((reverse_kernel<R, LW>), dim3((uint32_t)(1ull << P.n_glb)), dim3(1 << LW), lds, s, psi, lam,
                       plan.d_parts, pidx, plan.d_stages, plan.d_ops, plan.d_pool, gpart, stride);
    return hipGetLastError();
}

hipError_t launch_reverse(const Plan &plan, int R, int LW, int pidx, const float2 *psi, float2 *lam, double *gpart,
                          int64_t stride, hipStream_t s)
{
#define QSV_CASE(r, lw) \
    if (R == r && LW == lw) return launch_reverse_t<r, lw>(plan, pidx, psi, lam, gpart, stride, s);
    QSV_CASE(1, 6) QSV_CASE(2, 6) QSV_CASE(3, 6) QSV_CASE(4, 6) QSV_CASE(5, 6)
    QSV_CASE(3, 8) QSV_CASE(4, 8) QSV_CASE(5, 8) QSV_CASE(3, 9) QSV_CASE(4, 9) QSV_CASE(3, 10)
#undef QSV_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_grad_reduce(const Plan &plan, const double *gpart, int64_t n_slots, int64_t stride,
                              double *slot_sum, double *grad, hipStream_t s)
{
    if (n_slots > 0) {
        hipLaunchKernelGGL(slot_sum_kernel, dim3((uint32_t)n_slots), dim3(256), 0, s, gpart, stride, slot_sum);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t np = plan.n_params;
    hipLaunchKernelGGL(param_sum_kernel, dim3((uint32_t)((np + 255) / 256)), dim3(256), 0, s, plan.d_param_off,
                       plan.d_param_slots, slot_sum, np, grad);
    return hipGetLastError();
}

}  // namespace qsv
