// Expectation values of Pauli sums and the action of H on a state.
//
// A Pauli string P with X/Y mask xm and Z/Y mask zm maps |x> to
// i^{#Y} (-1)^{|x & zm|} |x ^ xm>, so
//   <psi|P|psi> = sum_x conj(psi_{x^xm}) psi_x i^{#Y} (-1)^{|x & zm|}.
// Terms are grouped by xm.  The groups, in increasing xm order, are cut into
// passes over the state: a pass has a set S of at most 12 tile qubits (qubits
// 0-3, for 128-byte runs, the X masks of its groups, then the lowest free
// qubits) and handles every group whose mask lies in S.  A workgroup reads a
// tile, the 2^|S| amplitudes with the other qubits fixed, into LDS, where the
// partner x ^ xm of each amplitude x then is; one pass reads the state once
// for all its groups.  (On the 20-qubit ansatz's H = sum Z_i Z_i+1 + sum X_i
// the 21 groups take two passes.)  A group whose mask does not fit a tile
// with the low qubits reads its partners from HBM.  Products are formed and
// accumulated in float64; block sums go to a partials array and a second
// kernel adds them in a fixed order, so results do not depend on timing.  (A
// last-workgroup-sums variant in one launch was slower: the release fence each
// workgroup needs before its ticket writes back its XCD's L2.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "gates.cuh"
#include "kernels.h"

namespace qsv {

constexpr int RED_THREADS = 256;

template <int THREADS = RED_THREADS>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double parity_sign(uint64_t v) { return (__popcll(v) & 1) ? -1.0 : 1.0; }

// A table record read by every lane alike (from LDS, into vector registers),
// moved to scalar registers: its fields then steer uniform branches and loops.
template <class T>
__device__ __forceinline__ T uniform(const T &x)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// One launch covers every pass: workgroup (x, pass, b) walks tiles x, x +
// gridDim.x, ... of state b with the pass's tile qubits.  A thread holds 8
// amplitudes of the tile (positions 2 tid + j + 1024 it, j < 2, it < 4), read
// as 16-byte pairs (qubit 0 is always a tile qubit).  Partner amplitudes
// of the pass's X/Y groups come from the LDS copy of the tile, those of wide
// groups (masks that do not fit a tile with the low qubits) from HBM.  The
// pass's group and term tables are copied to LDS first when they fit: on a
// small state a workgroup sees one tile, and reading them from memory group by
// group would put one memory latency per group on its critical path.
// partials[(b * n_passes + pass) * gridDim.x + block]
//
// Registers are capped at 128 per lane (4 waves per SIMD): two workgroups per
// compute unit, so one workgroup's tile load overlaps the other's arithmetic;
// at 3 waves per SIMD (one workgroup) the large-state pass lost a third of its
// bandwidth.
template <bool SMALL>
__global__ __launch_bounds__(EXPECT_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void expect_kernel(
    const DevPass *__restrict__ passes, int p0, int n_passes, const DevGroup *__restrict__ groups,
    const DevTerm *__restrict__ terms, int n, const float2 *__restrict__ psi, double *__restrict__ partials)
{
    typedef float nf4 __attribute__((ext_vector_type(4)));  // a vector type the builtin accepts
    __shared__ float4 lds4[(1 << EXPECT_TILE_QUBITS) / 2];
    __shared__ DevGroup s_groups[EXPECT_LDS_GROUPS];
    __shared__ DevTerm s_terms[EXPECT_LDS_TERMS];
    __shared__ double s_wave[EXPECT_THREADS / 64];
    const float2 *lds = reinterpret_cast<const float2 *>(lds4);
    const int pi = p0 + (int)blockIdx.y;
    const DevPass PS = passes[pi];
    const int64_t b = blockIdx.z;
    const float2 *__restrict__ s = psi + ((uint64_t)b << n);
    const uint32_t tid = threadIdx.x;
    const int t = n < EXPECT_TILE_QUBITS ? n : EXPECT_TILE_QUBITS;
    const uint32_t tdim = 1u << t;
    int t_base = 0;  // index of the pass's first term
    if (PS.staged) {
        const int ng = PS.g_end - PS.g_begin;
        t_base = groups[PS.g_begin].term_begin;
        const int nt = groups[PS.g_end - 1].term_end - t_base;
        for (int i = (int)tid; i < ng; i += EXPECT_THREADS) s_groups[i] = groups[PS.g_begin + i];
        for (int i = (int)tid; i < nt; i += EXPECT_THREADS) s_terms[i] = terms[t_base + i];
        __syncthreads();
    }
    // the qubit (as a one-bit mask) at each tile position, in increasing order
    uint64_t posbit[EXPECT_TILE_QUBITS];
    {
        uint64_t m = PS.tile_mask;
#pragma unroll
        for (int c = 0; c < EXPECT_TILE_QUBITS; ++c) {
            posbit[c] = m & (~m + 1);
            m &= m - 1;
        }
    }
    uint64_t xthr = 0;  // positions 2 tid: tile positions 1..LT
#pragma unroll
    for (int c = 1; c <= EXPECT_LOG_THREADS; ++c)
        if ((tid >> (c - 1)) & 1u) xthr |= posbit[c];
    uint64_t row[EXPECT_PAIRS];  // positions ROW it: the tile positions above
#pragma unroll
    for (int it = 0; it < EXPECT_PAIRS; ++it) {
        uint64_t r = 0;
#pragma unroll
        for (int c = EXPECT_LOG_THREADS + 1; c < EXPECT_TILE_QUBITS; ++c)
            if ((it >> (c - EXPECT_LOG_THREADS - 1)) & 1) r |= posbit[c];
        row[it] = r;
    }
    constexpr uint32_t ROW = 2u * EXPECT_THREADS;  // tile positions per pair row
    const uint64_t full = (1ull << n) - 1;
    const uint64_t outside = full & ~PS.tile_mask;
    const uint64_t n_tiles = 1ull << (n - t);
    double acc = 0.0;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        // the tile index's bits on the qubits outside the tile, in increasing order
        uint64_t base = 0, tl = tile;
        for (uint64_t f = outside; f && tl; f &= f - 1, tl >>= 1)
            if (tl & 1) base |= f & (~f + 1);
        float4 v[EXPECT_PAIRS];
        uint64_t x[EXPECT_PAIRS];  // index of the pair's first amplitude (qubit 0 clear)
#pragma unroll
        for (int it = 0; it < EXPECT_PAIRS; ++it) {
            x[it] = base | xthr | row[it];
            v[it] = float4{0.f, 0.f, 0.f, 0.f};
            if (2 * tid + ROW * it < tdim) {
                if (SMALL) {  // a state that stays in the caches (read by several passes)
                    v[it] = *reinterpret_cast<const float4 *>(s + x[it]);
                } else {
                    const nf4 w = __builtin_nontemporal_load(reinterpret_cast<const nf4 *>(s + x[it]));
                    v[it] = float4{w.x, w.y, w.z, w.w};
                }
            }
        }
        if (PS.has_x) {
            __syncthreads();  // the previous tile's partner reads are done
#pragma unroll
            for (int it = 0; it < EXPECT_PAIRS; ++it)
                if (2 * tid + ROW * it < tdim) lds4[tid + EXPECT_THREADS * it] = v[it];
            __syncthreads();
        }
        // the pass's groups g0..g1 of the tables GP (group g at GP[g - g0]) and
        // TP (term k at TP[k - tb])
        auto walk = [&](const DevGroup *__restrict__ GP, const DevTerm *__restrict__ TP, int tb) {
            for (int g = 0; g < PS.g_end - PS.g_begin; ++g) {
                const DevGroup G = uniform(GP[g]);
                if (G.x_mask == 0) {
                    // diagonal group: the weight w(x) = sum_t c_t (-1)^{|x & z_t|} of
                    // each of the thread's 8 amplitudes.  With x = base | 2 tid | slot
                    // u (u's bits at tile positions 0, 10, 11), the sign splits into
                    // a per-thread part and chi_t(u) = (-1)^{|u & slot_t|}.  The terms
                    // come sorted by slot_t: a_S = sum of c_t (-1)^{|(base | 2 tid) &
                    // z_t|} over the terms with slot S, then w(u) += chi_S(u) a_S.
                    // A term costs a few vector instructions; each of the at most 8
                    // patterns, 8 additions.
                    double w[2 * EXPECT_PAIRS];
#pragma unroll
                    for (int u = 0; u < 2 * EXPECT_PAIRS; ++u) w[u] = 0.0;
                    auto flush = [&](int pat, double a) {
#pragma unroll
                        for (int u = 0; u < 2 * EXPECT_PAIRS; ++u) w[u] += (__popc(pat & u) & 1) ? -a : a;
                    };
                    int pat = -1;
                    double a = 0.0;
                    for (int k = G.term_begin; k < G.term_end; ++k) {
                        const DevTerm &T = TP[k - tb];
                        const int ts = __builtin_amdgcn_readfirstlane(T.slot);
                        if (ts != pat) {
                            if (pat >= 0) flush(pat, a);
                            pat = ts;
                            a = 0.0;
                        }
                        const uint32_t par = (__popcll(base & T.z_mask) + __popc((2u * tid) & T.zt)) & 1u;
                        a += par ? -T.cre : T.cre;
                    }
                    if (pat >= 0) flush(pat, a);
#pragma unroll
                    for (int it = 0; it < EXPECT_PAIRS; ++it) {
                        const double p0v = (double)v[it].x * v[it].x + (double)v[it].y * v[it].y;
                        const double p1v = (double)v[it].z * v[it].z + (double)v[it].w * v[it].w;
                        acc += p0v * w[2 * it] + p1v * w[2 * it + 1];
                    }
                } else if (G.xt >= 0) {
                    // partners in the tile: the pairs (p0, p1 = p0 ^ xt) of tile
                    // positions with bit lb of p0 clear; per term, with
                    // z = conj(psi_p1) psi_p0 and signs from the term's Z mask on the
                    // tile (zt) and outside it (base):  s0 Re[c z] + s1 Re[c conj(z)]
                    const uint32_t xt = (uint32_t)G.xt;
                    const int lb = __builtin_ctz(xt);
                    const uint32_t below = (1u << lb) - 1;
                    // f(p0, psi_p0, psi_p1) for every pair of the tile, in a fixed order;
                    // the 16-byte reads only on cached states, where the LDS reads
                    // weigh (a streamed state is bound by HBM, and the extra registers
                    // slowed its loads)
                    auto for_pairs = [&](auto &&f) __attribute__((always_inline)) {
                        if (SMALL && xt == 1u) {
                            // X on position 0 alone: the partner is the other half of the
                            // thread's own 16-byte pair
#pragma unroll
                            for (int it = 0; it < EXPECT_PAIRS; ++it)
                                if (2 * tid + ROW * it < tdim)
                                    f(2 * tid + ROW * it, float2{v[it].x, v[it].y}, float2{v[it].z, v[it].w});
                        } else if (SMALL && lb >= 1) {
                            // pairs k and k + 1 (k even) are the adjacent positions p0 and
                            // p0 + 1 and their partners: one 16-byte LDS read for each side
#pragma unroll
                            for (int i = 0; i < EXPECT_PAIRS / 2; ++i) {
                                const uint32_t k = 2u * (tid + (uint32_t)EXPECT_THREADS * i);
                                if (k >= (tdim >> 1)) continue;
                                const uint32_t q0 = ((k >> lb) << (lb + 1)) | (k & below);
                                const float4 a4 = lds4[q0 >> 1], c4 = lds4[(q0 ^ xt) >> 1];
                                f(q0, float2{a4.x, a4.y}, float2{c4.x, c4.y});
                                f(q0 | 1u, float2{a4.z, a4.w}, float2{c4.z, c4.w});
                            }
                        } else {
#pragma unroll
                            for (int i = 0; i < EXPECT_PAIRS; ++i) {
                                const uint32_t k = tid + (uint32_t)EXPECT_THREADS * i;
                                if (k >= (tdim >> 1)) continue;
                                const uint32_t q0 = ((k >> lb) << (lb + 1)) | (k & below);
                                f(q0, lds[q0], lds[q0 ^ xt]);
                            }
                        }
                    };
                    const DevTerm T0 = uniform(TP[G.term_begin - tb]);
                    // a single real X string (the common case) takes the 16-byte
                    // reads; any other group reads pair by pair, k = tid + 512 i
                    if (G.term_end - G.term_begin == 1 && T0.z_mask == 0 && T0.cim == 0.0) {
                        // one real X string: 2 c Re z summed over the pairs
                        double gz = 0.0;
                        for_pairs([&](uint32_t, float2 a, float2 c) __attribute__((always_inline)) {
                            gz += (double)c.x * a.x + (double)c.y * a.y;
                        });
                        acc += 2.0 * T0.cre * gz;
                        continue;
                    }
#pragma unroll
                    for (int i = 0; i < EXPECT_PAIRS; ++i) {
                        const uint32_t k = tid + (uint32_t)EXPECT_THREADS * i;
                        if (k >= (tdim >> 1)) continue;
                        const uint32_t q0 = ((k >> lb) << (lb + 1)) | (k & below);
                        const float2 a = lds[q0], c = lds[q0 ^ xt];
                        const double zr = (double)c.x * a.x + (double)c.y * a.y;
                        const double zi = (double)c.x * a.y - (double)c.y * a.x;
                        for (int q = G.term_begin; q < G.term_end; ++q) {
                            const DevTerm T = uniform(TP[q - tb]);
                            const uint32_t s0 = (__popc(q0 & T.zt) + __popcll(base & T.z_mask)) & 1u;
                            const uint32_t s1 = s0 ^ (__popc(xt & T.zt) & 1u);
                            const double re = T.cre * zr - T.cim * zi, rc = T.cre * zr + T.cim * zi;
                            acc += (s0 ? -re : re) + (s1 ? -rc : rc);
                        }
                    }
                } else {
                    // a wide group: partners from HBM, every amplitude x of the tile
                    //   sum_t Re[c_t (-1)^{|x & z_t|} conj(psi_{x ^ m}) psi_x]
#pragma unroll
                    for (int it = 0; it < EXPECT_PAIRS; ++it) {
                        if (2 * tid + ROW * it >= tdim) continue;
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const float2 a = j ? float2{v[it].z, v[it].w} : float2{v[it].x, v[it].y};
                            const uint64_t xj = x[it] | (uint64_t)j;
                            const float2 c = s[xj ^ G.x_mask];
                            const double zr = (double)c.x * a.x + (double)c.y * a.y;
                            const double zi = (double)c.x * a.y - (double)c.y * a.x;
                            for (int q = G.term_begin; q < G.term_end; ++q) {
                                const DevTerm T = uniform(TP[q - tb]);
                                acc += parity_sign(xj & T.z_mask) * (T.cre * zr - T.cim * zi);
                            }
                        }
                    }
                }
            }
        };
        if (PS.staged)
            walk(s_groups, s_terms, t_base);
        else
            walk(groups + PS.g_begin, terms, 0);
    }
    // the workgroup's sum: waves in order
    const double wv = wave_sum(acc);
    if ((tid & 63) == 0) s_wave[tid >> 6] = wv;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
#pragma unroll
        for (int i = 0; i < EXPECT_THREADS / 64; ++i) tot += s_wave[i];
        partials[((uint64_t)b * n_passes + pi) * gridDim.x + blockIdx.x] = tot;
    }
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

// c with its sign bit flipped where bit 31 of sb is set.
__device__ __forceinline__ float flipf(float c, uint32_t sb) { return __uint_as_float(__float_as_uint(c) ^ sb); }
__device__ __forceinline__ double flipd(double c, uint32_t sb)
{
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, c) ^ ((uint64_t)sb << 32));
}

// lam = H psi as apply_h_kernel, four amplitudes per thread (n >= 2): the four
// values x0 + j of qubits 0 and 1, read and written as two 16-byte words.  For
// a group with X mask m the partners are the four amplitudes at x0 ^ (m & ~3),
// in the order j ^ (m & 3); a term's sign at amplitude j is its sign at x0
// times (-1)^{|j & Z|}, so one term costs one parity per four amplitudes.  A
// group of one term puts its sign on the partner amplitudes; a longer group
// sums its terms per pattern Z & 3 first.  Group and term records are loaded
// once per four amplitudes.
__global__ __launch_bounds__(RED_THREADS) void apply_h4_kernel(const DevGroup *__restrict__ groups, int n_groups,
                                                                const DevTerm *__restrict__ terms, int n,
                                                                const float2 *__restrict__ psi,
                                                                float2 *__restrict__ lam,
                                                                double *__restrict__ partials)
{
    __shared__ double sh[RED_THREADS];
    const uint64_t nc = 1ull << (n - 2);
    const uint64_t stride = (uint64_t)gridDim.x * RED_THREADS;
    const float4 *__restrict__ psi4 = reinterpret_cast<const float4 *>(psi);
    float4 *__restrict__ lam4 = reinterpret_cast<float4 *>(lam);
    double acc = 0.0;
    for (uint64_t c = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; c < nc; c += stride) {
        const uint64_t x0 = c << 2;
        const float4 pa = psi4[2 * c], pb = psi4[2 * c + 1];
        const float2 p[4] = {{pa.x, pa.y}, {pa.z, pa.w}, {pb.x, pb.y}, {pb.z, pb.w}};
        double lr[4] = {0.0, 0.0, 0.0, 0.0}, li[4] = {0.0, 0.0, 0.0, 0.0};
        for (int g = 0; g < n_groups; ++g) {
            const DevGroup G = groups[g];
            const uint64_t xm = G.x_mask;
            const uint64_t y0 = x0 ^ (xm & ~3ull);
            const float4 qa = psi4[y0 >> 1], qb = psi4[(y0 >> 1) + 1];
            float2 r[4] = {{qa.x, qa.y}, {qa.z, qa.w}, {qb.x, qb.y}, {qb.z, qb.w}};
            if (xm & 1) {  // r[j] = partner of amplitude j = q[j ^ (m & 3)]
                float2 t = r[0]; r[0] = r[1]; r[1] = t;
                t = r[2]; r[2] = r[3]; r[3] = t;
            }
            if (xm & 2) {
                float2 t = r[0]; r[0] = r[2]; r[2] = t;
                t = r[1]; r[1] = r[3]; r[3] = t;
            }
            if (G.term_end - G.term_begin == 1) {
                const DevTerm T = terms[G.term_begin];
                const uint32_t sb0 = (uint32_t)(__popcll((x0 ^ xm) & T.z_mask) & 1) << 31;
                const uint32_t zl = (uint32_t)T.z_mask & 3u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t sb = sb0 ^ ((uint32_t)(__popc((uint32_t)j & zl) & 1) << 31);
                    const double qx = (double)flipf(r[j].x, sb), qy = (double)flipf(r[j].y, sb);
                    lr[j] += T.cre * qx - T.cim * qy;
                    li[j] += T.cre * qy + T.cim * qx;
                }
                continue;
            }
            double br[4] = {0.0, 0.0, 0.0, 0.0}, bi[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = G.term_begin; k < G.term_end; ++k) {
                const DevTerm T = terms[k];
                const uint32_t sb = (uint32_t)(__popcll((x0 ^ xm) & T.z_mask) & 1) << 31;
                const int pat = (int)(T.z_mask & 3u);
                const double ar = flipd(T.cre, sb), ai = flipd(T.cim, sb);
                if (pat == 0) br[0] += ar, bi[0] += ai;
                else if (pat == 1) br[1] += ar, bi[1] += ai;
                else if (pat == 2) br[2] += ar, bi[2] += ai;
                else br[3] += ar, bi[3] += ai;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double wr = 0.0, wi = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool neg = __builtin_popcount(j & q) & 1;
                    wr += neg ? -br[q] : br[q];
                    wi += neg ? -bi[q] : bi[q];
                }
                lr[j] += wr * r[j].x - wi * r[j].y;
                li[j] += wr * r[j].y + wi * r[j].x;
            }
        }
        lam4[2 * c] = float4{(float)lr[0], (float)li[0], (float)lr[1], (float)li[1]};
        lam4[2 * c + 1] = float4{(float)lr[2], (float)li[2], (float)lr[3], (float)li[3]};
#pragma unroll
        for (int j = 0; j < 4; ++j) acc += (double)p[j].x * lr[j] + (double)p[j].y * li[j];
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

int expect_blocks(int n)
{
    const int t = std::min(n, EXPECT_TILE_QUBITS);
    return (int)std::min<uint64_t>(1ull << (n - t), EXPECT_MAX_BLOCKS);
}

int plan_expect_passes(int n, DevGroup *groups, int n_groups, DevTerm *terms, DevPass *passes)
{
    const int t = std::min(n, EXPECT_TILE_QUBITS);
    const uint64_t low = (1ull << std::min(n, 4)) - 1;  // qubits 0-3: 128-byte runs of the state
    auto compress = [&](uint64_t S, uint64_t m) {     // m on the tile positions of S
        uint32_t r = 0;
        for (int q = 0, c = 0; q < n; ++q)
            if ((S >> q) & 1) {
                if ((m >> q) & 1) r |= 1u << c;
                ++c;
            }
        return r;
    };
    int np = 0, begin = 0;
    uint64_t S = 0;
    auto close = [&](int end) {
        for (int q = 0; q < n && __builtin_popcountll(S) < t; ++q) S |= 1ull << q;
        DevPass &P = passes[np++];
        P.tile_mask = S;
        P.g_begin = begin;
        P.g_end = end;
        P.has_x = 0;
        P.staged = 0;
        for (int g = begin; g < end; ++g) {
            DevGroup &G = groups[g];
            G.pad = 0;
            for (int k = G.term_begin; k < G.term_end; ++k) {
                DevTerm &T = terms[k];
                T.zt = G.xt < 0 ? 0u : compress(S, T.z_mask);
                // bits of zt at the positions of a thread's 8 amplitudes (0, 10, 11)
                T.slot = (int32_t)((T.zt & 1u) | ((T.zt >> 9) & 2u) | ((T.zt >> 9) & 4u));
            }
            if (G.x_mask == 0)  // diagonal: terms of equal slot pattern together
                std::stable_sort(terms + G.term_begin, terms + G.term_end,
                                 [](const DevTerm &a, const DevTerm &b) { return a.slot < b.slot; });
            if (G.xt < 0) continue;  // wide: partners from HBM
            G.xt = (int32_t)compress(S, G.x_mask);
        }
    };
    for (int g = 0; g < n_groups; ++g) {
        const uint64_t xm = groups[g].x_mask;
        const bool wide = __builtin_popcountll(low | xm) > t;
        groups[g].xt = wide ? -1 : 0;
        const uint64_t need = wide ? low : (low | xm);
        if (g > begin && __builtin_popcountll(S | need) > t) {
            close(g);
            begin = g;
            S = 0;
        }
        S |= need;
    }
    if (n_groups > 0) close(n_groups);
    // few tiles (small states): split passes by their groups, so that the
    // launch has EXPECT_MIN_BLOCKS workgroups; in place, last pass first (the
    // parts of pass p land at indices >= p)
    const int64_t blocks = (int64_t)expect_blocks(n) * np;
    if (np > 0 && blocks < EXPECT_MIN_BLOCKS) {
        const int want = (int)((EXPECT_MIN_BLOCKS + blocks - 1) / blocks);
        int total = 0;
        for (int p = 0; p < np; ++p) total += std::min(want, passes[p].g_end - passes[p].g_begin);
        int out = total;
        for (int p = np - 1; p >= 0; --p) {
            const DevPass P = passes[p];
            const int ng = P.g_end - P.g_begin, c = std::min(want, ng);
            out -= c;
            for (int i = 0; i < c; ++i) {
                DevPass &Q = passes[out + i];
                Q = P;
                Q.g_begin = P.g_begin + (int)((int64_t)ng * i / c);
                Q.g_end = P.g_begin + (int)((int64_t)ng * (i + 1) / c);
            }
        }
        np = total;
    }
    for (int p = 0; p < np; ++p) {
        DevPass &P = passes[p];
        P.has_x = 0;
        bool contiguous = true;  // the groups' terms form one run (they do for grouped sums)
        for (int g = P.g_begin; g < P.g_end; ++g) {
            if (groups[g].x_mask && groups[g].xt >= 0) P.has_x = 1;
            if (g > P.g_begin && groups[g].term_begin != groups[g - 1].term_end) contiguous = false;
        }
        const int nt = groups[P.g_end - 1].term_end - groups[P.g_begin].term_begin;
        P.staged = contiguous && P.g_end - P.g_begin <= EXPECT_LDS_GROUPS && nt <= EXPECT_LDS_TERMS;
    }
    return np;
}

hipError_t launch_expect(const DevPass *passes, int n_passes, const DevGroup *groups, const DevTerm *terms, int n,
                         int64_t batch, const float2 *psi, double *partials, double *out, hipStream_t s)
{
    if (n_passes == 0) {  // empty sum: zeros
        hipLaunchKernelGGL(final_sum_kernel, dim3((uint32_t)batch), dim3(RED_THREADS), 0, s, partials, 0, out);
        return hipGetLastError();
    }
    const int nb = expect_blocks(n);
    auto kernel = n <= EXPECT_CACHED_QUBITS ? expect_kernel<true> : expect_kernel<false>;
    const int64_t lim = 65535;  // grid y and z limits: passes and batches beyond them go in chunks
    for (int64_t b0 = 0; b0 < batch; b0 += lim) {
        const int64_t nz = std::min<int64_t>(lim, batch - b0);
        for (int p0 = 0; p0 < n_passes; p0 += (int)lim) {
            const int ny = (int)std::min<int64_t>(lim, n_passes - p0);
            hipLaunchKernelGGL(kernel, dim3(nb, ny, (uint32_t)nz), dim3(EXPECT_THREADS), 0, s, passes, p0, n_passes,
                               groups, terms, n, psi + ((uint64_t)b0 << n), partials + (uint64_t)b0 * n_passes * nb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(final_sum_kernel, dim3((uint32_t)batch), dim3(RED_THREADS), 0, s, partials, nb * n_passes, out);
    return hipGetLastError();
}

int apply_h_blocks(int n, int cap)
{
    // four amplitudes per thread (one below n = 2)
    const uint64_t per_thread = n >= 2 ? 4 : 1;
    const uint64_t b = std::max<uint64_t>(1, (1ull << n) / (per_thread * RED_THREADS));
    return (int)std::min<uint64_t>(b, (uint64_t)std::max(cap, 1));
}

hipError_t launch_apply_h(const DevGroup *groups, int n_groups, const DevTerm *terms, int n, const float2 *psi,
                          float2 *lam, double *partials, int n_blocks, double *energy, hipStream_t s)
{
    const int nb = apply_h_blocks(n, n_blocks);
    if (n >= 2)
        hipLaunchKernelGGL(apply_h4_kernel, dim3(nb), dim3(RED_THREADS), 0, s, groups, n_groups, terms, n, psi, lam,
                           partials);
    else
        hipLaunchKernelGGL(apply_h_kernel, dim3(nb), dim3(RED_THREADS), 0, s, groups, n_groups, terms, n, psi, lam,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RED_THREADS), 0, s, partials, nb, energy);
    return hipGetLastError();
}

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

}  // namespace qsv
