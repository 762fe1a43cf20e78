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
#include "tile.cuh"

namespace qsv {

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

// Register diagonals folded from parameterised RZ rotations: entry u of
// diagonal i is exp(i/2 sum_m (2 u_{slot m} - 1) theta_m).  One thread per
// diagonal: each member's e^{-i theta/2} from cos/sin in float64, the entries
// as products of those factors and their conjugates (float64), rounded to
// float32.
__global__ void materialize_diag_kernel(const ParamDiag *__restrict__ pd, int n, int na,
                                        const double *__restrict__ theta, float *__restrict__ pool)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ParamDiag d = pd[i];
    double zr[MAX_R], zi[MAX_R];  // e^{-i theta_m / 2}
    for (int m = 0; m < d.n; ++m) {
        double s, c;
        sincos(0.5 * theta[d.theta[m]], &s, &c);
        zr[m] = c;
        zi[m] = -s;
    }
    float2 *out = reinterpret_cast<float2 *>(pool + d.mat);
    for (int u = 0; u < na; ++u) {
        double er = 1.0, ei = 0.0;
        for (int m = 0; m < d.n; ++m) {
            const double fi = ((u >> d.slot[m]) & 1) ? -zi[m] : zi[m];  // bit set: the conjugate
            const double r = er * zr[m] - ei * fi;
            ei = er * fi + ei * zr[m];
            er = r;
        }
        out[u] = float2{(float)er, (float)ei};
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
    if (!plan.spec_fn.empty() && plan.spec_fn[pidx]) {  // the partition's specialised kernel
        const float *pool = plan.d_pool;
        void *args[] = {&psi, &ckpt, &pool};
        return hipModuleLaunchKernel((hipFunction_t)plan.spec_fn[pidx], (uint32_t)tiles, 1, 1, 1u << LW, 1, 1,
                                     (uint32_t)lds, s, args, nullptr);
    }
    hipLaunchKernelGGL((sweep_kernel<R, LW>), dim3((uint32_t)tiles), dim3(1 << LW), lds, s, psi, ckpt,
                       plan.d_parts, pidx, plan.d_stages, plan.d_ops, plan.d_pool);
    return hipGetLastError();
}

bool kernel_shape_supported(int R, int LW)
{
    return (LW == 6 && R >= 1 && R <= 5) || (LW == 8 && R >= 3 && R <= 5) || (LW == 9 && R >= 3 && R <= 5) ||
           (LW == 10 && (R == 3 || R == 4));
}

hipError_t launch_sweep(const Plan &plan, int R, int LW, int pidx, float2 *psi, float2 *ckpt, hipStream_t s)
{
#define QSV_CASE(r, lw) \
    if (R == r && LW == lw) return launch_sweep_t<r, lw>(plan, pidx, psi, ckpt, s);
    QSV_CASE(1, 6) QSV_CASE(2, 6) QSV_CASE(3, 6) QSV_CASE(4, 6) QSV_CASE(5, 6)
    QSV_CASE(3, 8) QSV_CASE(4, 8) QSV_CASE(5, 8)
    QSV_CASE(3, 9) QSV_CASE(4, 9) QSV_CASE(5, 9) QSV_CASE(3, 10) QSV_CASE(4, 10)
#undef QSV_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_materialize(const Plan &plan, const double *theta, hipStream_t s, bool diags)
{
    const int n = (int)plan.pgates.size();
    if (n > 0) {
        hipLaunchKernelGGL(materialize_kernel, dim3((n + 255) / 256), dim3(256), 0, s, plan.d_pgates, n, theta,
                           plan.d_pool);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nd = (int)plan.pdiags.size(), na = 1 << plan.R;
    if (nd > 0 && diags) {
        hipLaunchKernelGGL(materialize_diag_kernel, dim3((uint32_t)((nd + 255) / 256)), dim3(256), 0, s,
                           plan.d_pdiags, nd, na, theta, plan.d_pool);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace qsv
