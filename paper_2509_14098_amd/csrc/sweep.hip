// Fused partition sweep (paper Section 4.3): one launch applies all gates of
// one partition to every tile of the state.
//
// Per workgroup (one tile of 2^t amplitudes: the partition's t tile qubits
// vary, the other n - t qubits are fixed by the tile index):
//   1. HBM -> LDS: 16-byte loads of amplitude pairs (tile position 0 is qubit
//      0, so each pair is contiguous in HBM); runs of 2^c contiguous
//      amplitudes where the c lowest qubits are in the tile;
//   2. for every register stage: LDS -> registers in the stage layout, the
//      stage's gates in registers, registers -> LDS, barrier;
//   3. LDS -> HBM (and, when asked, the same tile to the checkpoint buffer).
// The LDS tile is XOR-swizzled (swz) against bank conflicts.
#include <hip/hip_runtime.h>

#include "gates.cuh"
#include "kernels.h"

namespace qsv {

// Global amplitude offset of canonical tile bits [lo, hi) of c.
__device__ __forceinline__ uint64_t tile_offset(const DevPart *__restrict__ P, uint32_t c, int lo, int hi)
{
    uint64_t g = 0;
    for (int b = lo; b < hi; ++b)
        if ((c >> b) & 1u) g |= 1ull << P->tq[b];
    return g;
}

template <int R, int LW>
__device__ __forceinline__ uint64_t tile_base(const DevPart *__restrict__ P, uint64_t tile)
{
    uint64_t base = 0;
    for (int b = 0; b < P->n_glb; ++b)
        if ((tile >> b) & 1ull) base |= 1ull << P->gq[b];
    return base;
}

// Uniform HBM offsets of the pair rows handled in iteration it: bits of it
// sit at canonical tile positions LW+1, LW+2, ...
template <int ITER, int LW>
__device__ __forceinline__ void row_offsets(const DevPart *__restrict__ P, uint64_t (&g)[ITER])
{
    g[0] = 0;
#pragma unroll
    for (int it = 1; it < ITER; ++it) g[it] = g[it & (it - 1)] | (1ull << P->tq[LW + 1 + __builtin_ctz(it)]);
}

// Load the tile HBM -> LDS.  Pair p covers canonical positions 2p, 2p+1 (an
// aligned 16-byte pair in HBM, since tile position 0 is qubit 0).  A full
// tile (t = R + LW) issues all of a thread's loads before the LDS writes.
// Tiles that share no 128-byte line with another tile (every qubit below 4 is
// a tile qubit) are read with non-temporal loads: nothing else will use those
// lines.  Tiles that do share lines read through L2, where the neighbouring
// tiles (same XCD, see xcd_tile) find them.
template <int R, int LW>
__device__ __forceinline__ void load_tile(const float2 *__restrict__ psi, float2 *lds, const DevPart *__restrict__ P,
                                          uint64_t base, uint32_t tid)
{
    const int t = P->t;
    const int thr_hi = (LW + 1 < t) ? LW + 1 : t;
    const uint64_t gthr = base | tile_offset(P, 2u * tid, 1, thr_hi);
    if (t == R + LW) {
        constexpr int ITER = 1 << (R - 1);
        uint64_t g[ITER];
        row_offsets<ITER, LW>(P, g);
        float4 v[ITER];
        if (P->n_glb == 0 || P->gq[0] >= 4) {
            typedef float nf4 __attribute__((ext_vector_type(4)));  // a vector type the builtin accepts
#pragma unroll
            for (int it = 0; it < ITER; ++it) {
                const nf4 w = __builtin_nontemporal_load(reinterpret_cast<const nf4 *>(psi + (gthr | g[it])));
                v[it] = float4{w.x, w.y, w.z, w.w};
            }
        } else {
#pragma unroll
            for (int it = 0; it < ITER; ++it) v[it] = *reinterpret_cast<const float4 *>(psi + (gthr | g[it]));
        }
        const uint32_t st = swz(2u * tid);  // swz is linear and leaves bit 0 alone
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const uint32_t sc = st ^ swz(2u * (uint32_t)(it << LW));
            lds[sc] = float2{v[it].x, v[it].y};
            lds[sc ^ 1u] = float2{v[it].z, v[it].w};
        }
        return;
    }
    const uint32_t npairs = 1u << (t - 1);
    for (uint32_t p0 = 0; p0 < npairs; p0 += (1u << LW)) {
        const uint32_t p = p0 + tid;
        if (p < npairs) {
            const uint64_t g = gthr | tile_offset(P, 2u * p0, LW + 1, t);
            const float4 v = *reinterpret_cast<const float4 *>(psi + g);
            const uint32_t c = 2u * p;
            lds[swz(c)] = float2{v.x, v.y};
            lds[swz(c + 1)] = float2{v.z, v.w};
        }
    }
}

template <int R, int LW>
__device__ __forceinline__ void store_tile(float2 *__restrict__ psi, float2 *__restrict__ ckpt, const float2 *lds,
                                           const DevPart *__restrict__ P, uint64_t base, uint32_t tid)
{
    const int t = P->t;
    const int thr_hi = (LW + 1 < t) ? LW + 1 : t;
    const uint64_t gthr = base | tile_offset(P, 2u * tid, 1, thr_hi);
    if (t == R + LW) {
        constexpr int ITER = 1 << (R - 1);
        uint64_t g[ITER];
        row_offsets<ITER, LW>(P, g);
        float4 v[ITER];
        const uint32_t st = swz(2u * tid);
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const uint32_t sc = st ^ swz(2u * (uint32_t)(it << LW));
            const float2 x = lds[sc], y = lds[sc ^ 1u];
            v[it] = float4{x.x, x.y, y.x, y.y};
        }
        if (P->n_glb == 0 || P->gq[0] >= 4) {  // no shared lines: non-temporal stores too
            typedef float nf4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int it = 0; it < ITER; ++it)
                __builtin_nontemporal_store(nf4{v[it].x, v[it].y, v[it].z, v[it].w},
                                            reinterpret_cast<nf4 *>(psi + (gthr | g[it])));
        } else {
#pragma unroll
            for (int it = 0; it < ITER; ++it) *reinterpret_cast<float4 *>(psi + (gthr | g[it])) = v[it];
        }
        if (ckpt) {
#pragma unroll
            for (int it = 0; it < ITER; ++it) *reinterpret_cast<float4 *>(ckpt + (gthr | g[it])) = v[it];
        }
        return;
    }
    const uint32_t npairs = 1u << (t - 1);
    for (uint32_t p0 = 0; p0 < npairs; p0 += (1u << LW)) {
        const uint32_t p = p0 + tid;
        if (p < npairs) {
            const uint64_t g = gthr | tile_offset(P, 2u * p0, LW + 1, t);
            const uint32_t c = 2u * p;
            const float2 x = lds[swz(c)], y = lds[swz(c + 1)];
            const float4 v{x.x, x.y, y.x, y.y};
            *reinterpret_cast<float4 *>(psi + g) = v;
            if (ckpt) *reinterpret_cast<float4 *>(ckpt + g) = v;
        }
    }
}

template <int R, int LW>
__global__ __launch_bounds__(1 << LW) void sweep_kernel(float2 *__restrict__ psi, float2 *__restrict__ ckpt,
                                                          const DevPart *__restrict__ parts, int pidx,
                                                          const DevStage *__restrict__ stages,
                                                          const DevOp *__restrict__ ops,
                                                          const float *__restrict__ pool)
{
    extern __shared__ float2 lds[];
    const DevPart *__restrict__ P = parts + pidx;
    const uint32_t tid = threadIdx.x;
    const uint64_t base = tile_base<R, LW>(P, xcd_tile(blockIdx.x, gridDim.x, P));
    load_tile<R, LW>(psi, lds, P, base, tid);
    __syncthreads();
    run_stages<R, false>(lds, stages, ops, pool, P->stage_begin, P->stage_end, P->t - R, tid, base);
    store_tile<R, LW>(psi, ckpt, lds, P, base, tid);
}

// Rotation matrices from theta: cos/sin in float64, rounded to float32.
__global__ void materialize_kernel(const ParamGate *__restrict__ pg, int n, const double *__restrict__ theta,
                                   float *__restrict__ pool)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ParamGate g = pg[i];
    const double a = theta[g.theta_index];
    double s, c;
    sincos(0.5 * a, &s, &c);
    float *m = pool + g.mat;
    for (int k = 0; k < 8; ++k) m[k] = 0.f;
    switch (g.kind) {
    case QSV_RX:  // [[c, -i s], [-i s, c]]
        m[0] = (float)c; m[3] = (float)-s; m[5] = (float)-s; m[6] = (float)c; break;
    case QSV_RY:  // [[c, -s], [s, c]]
        m[0] = (float)c; m[2] = (float)-s; m[4] = (float)s; m[6] = (float)c; break;
    case QSV_RZ:  // diag(e^{-ia/2}, e^{ia/2}) as a full 2x2
        m[0] = (float)c; m[1] = (float)-s; m[6] = (float)c; m[7] = (float)s; break;
    default:      // RZZ: diagonal entries j = b(q0) + 2 b(q1): even parity e^{-ia/2}
        m[0] = (float)c; m[1] = (float)-s; m[2] = (float)c; m[3] = (float)s;
        m[4] = (float)c; m[5] = (float)s; m[6] = (float)c; m[7] = (float)-s; break;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <int R, int LW>
static hipError_t launch_sweep_t(const Plan &plan, int pidx, float2 *psi, float2 *ckpt, hipStream_t s)
{
    const DevPart &P = plan.parts[pidx];
    const size_t lds = (size_t)8 << P.t;
    static bool attr = false;
    if (!attr) {  // allow the full 160 KiB of LDS (advisory: ignored where not needed)
        (void)hipFuncSetAttribute((const void *)sweep_kernel<R, LW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipGetLastError();
        attr = true;
    }
    const uint64_t tiles = 1ull << P.n_glb;
    hipLaunchKernelGGL((sweep_kernel<R, LW>), dim3((uint32_t)tiles), dim3(1 << LW), lds, s, psi, ckpt,
                       plan.d_parts, pidx, plan.d_stages, plan.d_ops, plan.d_pool);
    return hipGetLastError();
}

bool kernel_shape_supported(int R, int LW)
{
    return (LW == 6 && R >= 1 && R <= 5) || (LW == 8 && R >= 3 && R <= 5) || (LW == 9 && (R == 4 || R == 5)) || (LW == 10 && R == 4);
}

hipError_t launch_sweep(const Plan &plan, int R, int LW, int pidx, float2 *psi, float2 *ckpt, hipStream_t s)
{
#define QSV_CASE(r, lw) \
    if (R == r && LW == lw) return launch_sweep_t<r, lw>(plan, pidx, psi, ckpt, s);
    QSV_CASE(1, 6) QSV_CASE(2, 6) QSV_CASE(3, 6) QSV_CASE(4, 6) QSV_CASE(5, 6)
    QSV_CASE(3, 8) QSV_CASE(4, 8) QSV_CASE(5, 8)
    QSV_CASE(4, 9) QSV_CASE(5, 9) QSV_CASE(4, 10)
#undef QSV_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_materialize(const Plan &plan, const double *theta, hipStream_t s)
{
    const int n = (int)plan.pgates.size();
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(materialize_kernel, dim3((n + 255) / 256), dim3(256), 0, s, plan.d_pgates, n, theta,
                       plan.d_pool);
    return hipGetLastError();
}

}  // namespace qsv
