// Tile staging between HBM and LDS for the partition sweeps (paper Section
// 4.3: the state is split on the partition's global qubits into tiles, and
// each tile is packed into on-chip memory, updated and written back).
//
// A tile holds 2^t amplitudes: the partition's t tile qubits vary, the other
// n - t qubits are fixed by the tile index.  Tile position 0 is always qubit
// 0, so amplitude pairs (2p, 2p+1) are 16 contiguous bytes in HBM.  The LDS
// copy is XOR-swizzled (swz) against bank conflicts.
#pragma once
#ifndef __HIPCC_RTC__  // hipRTC provides the runtime declarations itself
#include <hip/hip_runtime.h>
#endif

#include "gates.cuh"

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

// Tile copies HBM -> LDS and LDS -> HBM for the adjoint walk, one amplitude
// pair per thread per step (any tile size).
template <int LW>
__device__ __forceinline__ void load_pairs(const float2 *__restrict__ src, float2 *lds, const DevPart *__restrict__ P,
                                           uint64_t base, uint32_t tid)
{
    const int t = P->t;
    const uint32_t npairs = 1u << (t - 1);
    uint64_t gthr = 0;
    for (int b = 1; b < LW + 1 && b < t; ++b)
        if (((2u * tid) >> b) & 1u) gthr |= 1ull << P->tq[b];
    for (uint32_t p0 = 0; p0 < npairs; p0 += (1u << LW)) {
        const uint32_t p = p0 + tid;
        if (p < npairs) {
            uint64_t g = base | gthr;
            for (int b = LW + 1; b < t; ++b)
                if (((2u * p0) >> b) & 1u) g |= 1ull << P->tq[b];
            const float4 v = *reinterpret_cast<const float4 *>(src + g);
            lds[swz(2u * p)] = float2{v.x, v.y};
            lds[swz(2u * p + 1)] = float2{v.z, v.w};
        }
    }
}

template <int LW>
__device__ __forceinline__ void store_pairs(float2 *__restrict__ dst, const float2 *lds, const DevPart *__restrict__ P,
                                            uint64_t base, uint32_t tid)
{
    const int t = P->t;
    const uint32_t npairs = 1u << (t - 1);
    uint64_t gthr = 0;
    for (int b = 1; b < LW + 1 && b < t; ++b)
        if (((2u * tid) >> b) & 1u) gthr |= 1ull << P->tq[b];
    for (uint32_t p0 = 0; p0 < npairs; p0 += (1u << LW)) {
        const uint32_t p = p0 + tid;
        if (p < npairs) {
            uint64_t g = base | gthr;
            for (int b = LW + 1; b < t; ++b)
                if (((2u * p0) >> b) & 1u) g |= 1ull << P->tq[b];
            const float2 x = lds[swz(2u * p)], y = lds[swz(2u * p + 1)];
            *reinterpret_cast<float4 *>(dst + g) = float4{x.x, x.y, y.x, y.y};
        }
    }
}

}  // namespace qsv
