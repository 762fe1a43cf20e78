// Partition sweeps specialised for one plan (paper Section 4.3, Step D: the
// paper generates the computation of every partition as code).  The host
// emits, per partition, constexpr tables at namespace scope, a table type T
// that refers to them, and one kernel that calls spec_sweep<T>:
//
//   T::R, T::LW         register qubits and log2 threads of the plan's shape
//   T::part             the partition's DevPart (tile qubits, tile-index bits)
//   T::stages[]         its register stages, op ranges local to T::ops
//   T::ops[]            its lowered ops; mat indexes T::pool, or the device
//                       matrix pool where T::dyn[k] is set (matrices formed
//                       from theta at apply time)
//   T::pool[]           the constant matrices, diagonals and shear parameters
//
// The sweep is the same as sweep_kernel's: tile HBM -> LDS, register stages,
// LDS -> HBM, with the same gate bodies.  With every op known at compile
// time the op dispatch (kind and slot tests, table loads, branches) folds
// away and the gate constants become scalar operands.
#pragma once
#ifndef __HIPCC_RTC__  // hipRTC provides the runtime declarations itself
#include <hip/hip_runtime.h>
#endif

#include "gates.cuh"
#include "tile.cuh"

namespace qsv {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(IC<B>{});
        static_for<B + 1, E>(static_cast<F &&>(f));
    }
}

// Op K of T on one thread's amplitudes (forward direction).
template <class T, int K>
__device__ __forceinline__ void spec_op(float2 (&a)[1 << T::R], const float *__restrict__ dpool, uint32_t tid,
                                        uint64_t base)
{
    constexpr int R = T::R;
    constexpr DevOp o = T::ops[K];
    constexpr int ja = o.a & 0x3F, jb = o.b & 0x3F;
    const float *__restrict__ m = T::dyn[K] ? dpool + o.mat : T::pool + (o.mat < 0 ? 0 : o.mat);
    if constexpr (o.kind == OP_LAYER) {
        g_layer<R, false>(a, m, (uint32_t)o.a);
    } else if constexpr (o.kind == OP_DREG) {
        g_dreg<R, false>(a, m);
    } else if constexpr (o.kind == OP_CZ_RT) {
        static_assert(ja < R, "register slot");
        g_cz_rt<R, ja>(a, lane_bit(o.b, tid, base) << 31);
    } else if constexpr (o.kind == OP_CZ_TT) {
        g_cz_tt<R>(a, (lane_bit(o.a, tid, base) & lane_bit(o.b, tid, base)) << 31);
    } else if constexpr (o.kind == OP_CX) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        g_cx_reg<R, ja, jb>(a);
    } else if constexpr (o.kind == OP_CX_T) {
        static_assert(jb < R, "register slot");
        g_cx_lane<R, jb>(a, 0u - lane_bit(o.a, tid, base));
    } else if constexpr (o.kind == OP_U1) {
        static_assert(ja < R, "register slot");
        g_u1<R, ja, false>(a, m);
    } else if constexpr (o.kind == OP_R1) {
        static_assert(ja < R, "register slot");
        g_r1<R, ja, false>(a, m);
    } else if constexpr (o.kind == OP_CZ) {
        g_cz<R>(a, reg_pattern(ja) & reg_pattern(jb));
    } else if constexpr (o.kind == OP_D1) {
        static_assert(ja < R, "register slot");
        g_d1<R, ja, false>(a, m);
    } else if constexpr (o.kind == OP_D1_T) {
        g_d1_lane<R, false>(a, m, lane_bit(o.a, tid, base));
    } else if constexpr (o.kind == OP_D2) {
        g_d2<R, false>(a, m, loc_pattern(o.a, tid, base), loc_pattern(o.b, tid, base));
    } else if constexpr (o.kind == OP_D2_RT) {
        static_assert(ja < R, "register slot");
        g_d2_rt<R, ja, false>(a, m, lane_bit(o.b, tid, base), o.flags & 1);
    } else if constexpr (o.kind == OP_D2_TT) {
        g_d2_tt<R, false>(a, m, lane_bit(o.a, tid, base) + 2u * lane_bit(o.b, tid, base));
    } else if constexpr (o.kind == OP_CU) {
        static_assert(jb < R, "register slot");
        g_cu<R, jb, false>(a, m, loc_pattern(o.a, tid, base));
    } else if constexpr (o.kind == OP_U2) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        g_u2<R, ja, jb, false>(a, m);
    } else if constexpr (o.kind == OP_SWAP) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        g_swap<R, ja, jb>(a);
    } else {
        static_assert(o.kind == OP_LAYER, "unknown op kind");
    }
}

// Register stage S of T: LDS -> registers, its ops, registers -> LDS, barrier.
template <class T, int S>
__device__ __forceinline__ void spec_stage(float2 *lds, const float *__restrict__ dpool, uint32_t tid, uint64_t base)
{
    constexpr int R = T::R, NA = 1 << R, w = T::part.t - R;
    if (w == T::LW || tid < (1u << w)) {
        uint32_t toff, roff[NA];
        stage_offsets<R>(&T::stages[S], w, tid, toff, roff);
        float2 a[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) a[i] = lds[toff ^ roff[i]];
        static_for<T::stages[S].op_begin, T::stages[S].op_end>([&](auto K) __attribute__((always_inline)) {
            spec_op<T, std::decay_t<decltype(K)>::value>(a, dpool, tid, base);
        });
        asm volatile("" : "+v"(toff));  // recompute the write-back addresses instead of keeping 2^R live
#pragma unroll
        for (int i = 0; i < NA; ++i) lds[toff ^ roff[i]] = a[i];
    }
    __syncthreads();
}

// One workgroup per tile, as in sweep_kernel.
template <class T>
__device__ __forceinline__ void spec_sweep(float2 *__restrict__ psi, float2 *__restrict__ ckpt,
                                           const float *__restrict__ dpool)
{
    extern __shared__ float2 lds[];
    const DevPart *__restrict__ P = &T::part;
    const uint32_t tid = threadIdx.x;
    const uint64_t base = tile_base<T::R, T::LW>(P, xcd_tile(blockIdx.x, gridDim.x, P));
    load_tile<T::R, T::LW>(psi, lds, P, base, tid);
    __syncthreads();
    static_for<T::part.stage_begin, T::part.stage_end>([&](auto S) __attribute__((always_inline)) {
        spec_stage<T, std::decay_t<decltype(S)>::value>(lds, dpool, tid, base);
    });
    store_tile<T::R, T::LW>(psi, ckpt, lds, P, base, tid);
}

}  // namespace qsv
