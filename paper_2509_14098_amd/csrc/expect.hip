// Expectation values of Pauli sums and the action of H on a state.
//
// A Pauli string P with X/Y mask xm and Z/Y mask zm maps |x> to
// i^{#Y} (-1)^{|x & zm|} |x ^ xm>, so
//   <psi|P|psi> = sum_x conj(psi_{x^xm}) psi_x i^{#Y} (-1)^{|x & zm|}.
// Terms are grouped by xm; a group with xm != 0 is summed over pairs
// (x, x^xm), each amplitude read once per group.  Products are formed and
// accumulated in float64; block sums go to a partials array and a second
// kernel adds them in a fixed order, so results do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace qsv {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double parity_sign(uint64_t v) { return (__popcll(v) & 1) ? -1.0 : 1.0; }

// partials[(b * n_groups + g) * gridDim.x + block] for the groups g = g0 + blockIdx.y
__global__ __launch_bounds__(RED_THREADS) void expect_kernel(const DevGroup *__restrict__ groups, int g0,
                                                              int n_groups, const DevTerm *__restrict__ terms, int n,
                                                              const float2 *__restrict__ psi,
                                                              double *__restrict__ partials)
{
    __shared__ double sh[RED_THREADS];
    const int gi = g0 + (int)blockIdx.y;
    const int64_t b = blockIdx.z;
    const DevGroup G = groups[gi];
    const float2 *__restrict__ s = psi + ((uint64_t)b << n);
    const uint64_t stride = (uint64_t)gridDim.x * RED_THREADS;
    double acc = 0.0;
    if (G.x_mask == 0) {
        // diagonal group: amplitudes read as 16-byte pairs, eight pairs in flight per
        // thread, with non-temporal loads (the state is read once)
        auto weight = [&](uint64_t x) __attribute__((always_inline)) {
            double w = 0.0;
            for (int t = G.term_begin; t < G.term_end; ++t) w += terms[t].cre * parity_sign(x & terms[t].z_mask);
            return w;
        };
        auto pair = [&](uint64_t i, float4 v) __attribute__((always_inline)) {
            const double p0 = (double)v.x * v.x + (double)v.y * v.y, p1 = (double)v.z * v.z + (double)v.w * v.w;
            return p0 * weight(2 * i) + p1 * weight(2 * i + 1);
        };
        if (n == 1) {
            if (blockIdx.x == 0 && threadIdx.x == 0) acc = pair(0, *reinterpret_cast<const float4 *>(s));
        } else {
            const uint64_t n2 = 1ull << (n - 1);
            const float4 *__restrict__ s4 = reinterpret_cast<const float4 *>(s);
            uint64_t i = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x;
            for (; i + 7 * stride < n2; i += 8 * stride) {
                typedef float nf4 __attribute__((ext_vector_type(4)));  // a vector type the builtin accepts
                const nf4 *__restrict__ n4 = reinterpret_cast<const nf4 *>(s4);
                nf4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(n4 + i + u * stride);
                // the 16 weights with the term loop outside: 16 independent float64
                // sums per term (one chain per amplitude would leave the lanes
                // waiting on each add); each weight still adds its terms in order
                double w[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) w[u] = 0.0;
                for (int t = G.term_begin; t < G.term_end; ++t) {
                    const double c = terms[t].cre;
                    const uint64_t zm = terms[t].z_mask;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const uint64_t x = 2 * (i + u * stride);
                        w[2 * u] += c * parity_sign(x & zm);
                        w[2 * u + 1] += c * parity_sign((x + 1) & zm);
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double p0 = (double)v[u].x * v[u].x + (double)v[u].y * v[u].y;
                    const double p1 = (double)v[u].z * v[u].z + (double)v[u].w * v[u].w;
                    acc += p0 * w[2 * u] + p1 * w[2 * u + 1];
                }
            }
            for (; i < n2; i += stride) acc += pair(i, s4[i]);
        }
    } else {
        const int lb = __builtin_ctzll(G.x_mask);
        const uint64_t low = 1ull << lb;
        const uint64_t half = 1ull << (n - 1);
        auto term_sum = [&](uint64_t x, float2 a, float2 c) __attribute__((always_inline)) {
            const uint64_t y = x ^ G.x_mask;
            // z = conj(psi_y) psi_x
            const double zr = (double)c.x * a.x + (double)c.y * a.y;
            const double zi = (double)c.x * a.y - (double)c.y * a.x;
            for (int t = G.term_begin; t < G.term_end; ++t) {
                const DevTerm T = terms[t];
                const double sx = parity_sign(x & T.z_mask), sy = parity_sign(y & T.z_mask);
                acc += sx * (T.cre * zr - T.cim * zi) + sy * (T.cre * zr + T.cim * zi);
            }
        };
        auto first = [&](uint64_t k) __attribute__((always_inline)) { return ((k >> lb) << (lb + 1)) | (k & (low - 1)); };
        uint64_t k = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x;
        // four pairs' loads in flight per thread, then their sums in the order of the plain loop
        for (; k + 3 * stride < half; k += 4 * stride) {
            float2 a[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t x = first(k + u * stride);
                a[u] = s[x];
                c[u] = s[x ^ G.x_mask];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) term_sum(first(k + u * stride), a[u], c[u]);
        }
        for (; k < half; k += stride) {
            const uint64_t x = first(k);
            term_sum(x, s[x], s[x ^ G.x_mask]);
        }
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[((uint64_t)b * n_groups + gi) * gridDim.x + blockIdx.x] = tot;
}

// out[b] = sum of per_batch partials, fixed order
__global__ __launch_bounds__(RED_THREADS) void final_sum_kernel(const double *__restrict__ partials, int per_batch,
                                                                 double *__restrict__ out)
{
    __shared__ double sh[RED_THREADS];
    const int64_t b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < per_batch; i += RED_THREADS) acc += partials[b * per_batch + i];
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) out[b] = tot;
}

// lam = H psi; partials[block] = sum_x Re(conj(psi_x) lam_x) over the block
__global__ __launch_bounds__(RED_THREADS) void apply_h_kernel(const DevGroup *__restrict__ groups, int n_groups,
                                                               const DevTerm *__restrict__ terms, int n,
                                                               const float2 *__restrict__ psi,
                                                               float2 *__restrict__ lam,
                                                               double *__restrict__ partials)
{
    __shared__ double sh[RED_THREADS];
    const uint64_t dim = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * RED_THREADS;
    double acc = 0.0;
    for (uint64_t x = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; x < dim; x += stride) {
        const float2 px = psi[x];
        double lr = 0.0, li = 0.0;
        auto add_group = [&](const DevGroup &G, float2 py) __attribute__((always_inline)) {
            const uint64_t y = x ^ G.x_mask;
            double wr = 0.0, wi = 0.0;
            for (int t = G.term_begin; t < G.term_end; ++t) {
                const double sg = parity_sign(y & terms[t].z_mask);
                wr += sg * terms[t].cre;
                wi += sg * terms[t].cim;
            }
            lr += wr * py.x - wi * py.y;
            li += wr * py.y + wi * py.x;
        };
        int g = 0;
        // four groups' gathers in flight, then their sums in group order
        for (; g + 3 < n_groups; g += 4) {
            float2 py[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t xm = groups[g + u].x_mask;
                py[u] = xm ? psi[x ^ xm] : px;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) add_group(groups[g + u], py[u]);
        }
        for (; g < n_groups; ++g) {
            const uint64_t xm = groups[g].x_mask;
            add_group(groups[g], xm ? psi[x ^ xm] : px);
        }
        lam[x] = float2{(float)lr, (float)li};
        acc += (double)px.x * lr + (double)px.y * li;
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

static int blocks_for(uint64_t work, int cap)
{
    uint64_t b = (work + RED_THREADS * 16 - 1) / (RED_THREADS * 16);
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, (uint64_t)cap));
}

int expect_blocks(int n, int cap) { return blocks_for(1ull << n, cap); }

// Scratch of qsv_expect_noalloc: one fixed array per device, in the code
// object's own device memory, so the entry point never allocates.  Host code
// reaches it only through the address hipGetSymbolAddress returns on each
// device (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static void *g_scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mutex;

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_dev[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the lookup is per device: that device must be current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_dev[device];
}

hipError_t launch_expect(const DevGroup *groups, int n_groups, const DevTerm *terms, int n, int64_t batch,
                         const float2 *psi, double *partials, int n_blocks, double *out, hipStream_t s)
{
    if (n_groups == 0) {  // empty sum: zeros
        hipLaunchKernelGGL(final_sum_kernel, dim3((uint32_t)batch), dim3(RED_THREADS), 0, s, partials, 0, out);
        return hipGetLastError();
    }
    const int nb = blocks_for(1ull << n, n_blocks);
    const int64_t lim = 65535;  // grid y and z limits: groups and batches beyond them go in chunks
    for (int64_t b0 = 0; b0 < batch; b0 += lim) {
        const int64_t nz = std::min<int64_t>(lim, batch - b0);
        for (int g0 = 0; g0 < n_groups; g0 += (int)lim) {
            const int ny = (int)std::min<int64_t>(lim, n_groups - g0);
            hipLaunchKernelGGL(expect_kernel, dim3(nb, ny, (uint32_t)nz), dim3(RED_THREADS), 0, s, groups, g0, n_groups,
                               terms, n, psi + ((uint64_t)b0 << n), partials + (uint64_t)b0 * n_groups * nb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(final_sum_kernel, dim3((uint32_t)batch), dim3(RED_THREADS), 0, s, partials, nb * n_groups, out);
    return hipGetLastError();
}

int apply_h_blocks(int n, int cap)
{
    // one amplitude per thread: each amplitude walks every Pauli group with a
    // dependent table load and gather, so many waves are needed to cover them
    const uint64_t b = std::max<uint64_t>(1, (1ull << n) / RED_THREADS);
    return (int)std::min<uint64_t>(b, (uint64_t)std::max(cap, 1));
}

hipError_t launch_apply_h(const DevGroup *groups, int n_groups, const DevTerm *terms, int n, const float2 *psi,
                          float2 *lam, double *partials, int n_blocks, double *energy, hipStream_t s)
{
    const int nb = apply_h_blocks(n, n_blocks);
    hipLaunchKernelGGL(apply_h_kernel, dim3(nb), dim3(RED_THREADS), 0, s, groups, n_groups, terms, n, psi, lam,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RED_THREADS), 0, s, partials, nb, energy);
    return hipGetLastError();
}

}  // namespace qsv
