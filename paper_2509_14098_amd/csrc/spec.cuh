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

#include "batched.cuh"
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

// Op K of T (DAG: its conjugate transpose) on one or more amplitude arrays of
// a thread.
template <class T, int K, bool DAG, typename... Arr>
__device__ __forceinline__ void spec_op(const float *__restrict__ dpool, uint32_t tid, uint64_t base, Arr &...a)
{
    constexpr int R = T::R;
    constexpr DevOp o = T::ops[K];
    constexpr int ja = o.a & 0x3F, jb = o.b & 0x3F;
    const float *__restrict__ m = T::dyn[K] ? dpool + o.mat : T::pool + (o.mat < 0 ? 0 : o.mat);
    if constexpr (o.kind == OP_LAYER) {
        (g_layer<R, DAG>(a, m, (uint32_t)o.a), ...);
    } else if constexpr (o.kind == OP_DREG) {
        (g_dreg<R, DAG>(a, m), ...);
    } else if constexpr (o.kind == OP_CZ_RT) {
        static_assert(ja < R, "register slot");
        const uint32_t sg = lane_bit(o.b, tid, base) << 31;
        (g_cz_rt<R, ja>(a, sg), ...);
    } else if constexpr (o.kind == OP_CZ_TT) {
        const uint32_t sg = (lane_bit(o.a, tid, base) & lane_bit(o.b, tid, base)) << 31;
        (g_cz_tt<R>(a, sg), ...);
    } else if constexpr (o.kind == OP_CX) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        (g_cx_reg<R, ja, jb>(a), ...);
    } else if constexpr (o.kind == OP_CX_T) {
        static_assert(jb < R, "register slot");
        const uint32_t mk = 0u - lane_bit(o.a, tid, base);
        (g_cx_lane<R, jb>(a, mk), ...);
    } else if constexpr (o.kind == OP_U1) {
        static_assert(ja < R, "register slot");
        (g_u1<R, ja, DAG>(a, m), ...);
    } else if constexpr (o.kind == OP_R1) {
        static_assert(ja < R, "register slot");
        (g_r1<R, ja, DAG>(a, m), ...);
    } else if constexpr (o.kind == OP_CZ) {
        (g_cz<R>(a, reg_pattern(ja) & reg_pattern(jb)), ...);
    } else if constexpr (o.kind == OP_D1) {
        static_assert(ja < R, "register slot");
        (g_d1<R, ja, DAG>(a, m), ...);
    } else if constexpr (o.kind == OP_D1_T) {
        const uint32_t bit = lane_bit(o.a, tid, base);
        (g_d1_lane<R, DAG>(a, m, bit), ...);
    } else if constexpr (o.kind == OP_D2) {
        const uint32_t pa = loc_pattern(o.a, tid, base), pb = loc_pattern(o.b, tid, base);
        (g_d2<R, DAG>(a, m, pa, pb), ...);
    } else if constexpr (o.kind == OP_D2_RT) {
        static_assert(ja < R, "register slot");
        const uint32_t bit = lane_bit(o.b, tid, base);
        (g_d2_rt<R, ja, DAG>(a, m, bit, o.flags & 1), ...);
    } else if constexpr (o.kind == OP_D2_TT) {
        const uint32_t j = lane_bit(o.a, tid, base) + 2u * lane_bit(o.b, tid, base);
        (g_d2_tt<R, DAG>(a, m, j), ...);
    } else if constexpr (o.kind == OP_CU) {
        static_assert(jb < R, "register slot");
        const uint32_t pc = loc_pattern(o.a, tid, base);
        (g_cu<R, jb, DAG>(a, m, pc), ...);
    } else if constexpr (o.kind == OP_U2) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        (g_u2<R, ja, jb, DAG>(a, m), ...);
    } else if constexpr (o.kind == OP_SWAP) {
        static_assert(ja < R && jb < R && ja != jb, "register slots");
        (g_swap<R, ja, jb>(a), ...);
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
        for (int i = 0; i < NA; ++i) a[i] = lds_ref(lds, toff ^ roff[i]);
        static_for<T::stages[S].op_begin, T::stages[S].op_end>([&](auto K) __attribute__((always_inline)) {
            spec_op<T, std::decay_t<decltype(K)>::value, false>(dpool, tid, base, a);
        });
#pragma unroll
        for (int i = 0; i < NA; ++i) lds_ref(lds, toff ^ roff[i]) = a[i];
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

// Im <lambda|P|psi> over a thread's amplitudes for op K's generator P (the
// gradient term of a parameterised rotation exp(-i a P / 2)).
template <class T, int K>
__device__ __forceinline__ double spec_grad(const float2 (&a)[1 << T::R], const float2 (&l)[1 << T::R], uint32_t tid,
                                            uint64_t base)
{
    constexpr int R = T::R;
    constexpr DevOp o = T::ops[K];
    constexpr int ja = o.a & 0x3F;
    if constexpr (o.gen == GEN_Z && (o.a & LOC_MASK) == LOC_REG) {
        return grad_z_reg<R, ja>(a, l);
    } else if constexpr (o.gen == GEN_Z || o.gen == GEN_ZZ) {
        uint32_t p = loc_pattern(o.a, tid, base);
        if constexpr (o.gen == GEN_ZZ) p ^= loc_pattern(o.b, tid, base);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) acc = acc_im(acc, ((p >> i) & 1u) ? float2{-l[i].x, -l[i].y} : l[i], a[i]);
        return acc;
    } else {
        static_assert(o.gen == GEN_X || o.gen == GEN_Y, "rotation generator");
        static_assert((o.a & LOC_MASK) == LOC_REG && ja < R, "register slot");
        return grad_pairs<R, ja, o.gen == GEN_Y>(a, l);
    }
}

// Register stage S of T walked backwards on psi and lambda: for every op, last
// to first, the gradient term of a parameterised rotation (per-wave float64
// sum to gpart), then the op's conjugate transpose on both states.
template <class T, int S>
__device__ __forceinline__ void spec_reverse_stage(float2 *lds_psi, float2 *lds_lam, const float *__restrict__ dpool,
                                                   double *__restrict__ gpart, int64_t slot_stride, int64_t part_index,
                                                   uint32_t tid, uint64_t base)
{
    constexpr int R = T::R, NA = 1 << R, w = T::part.t - R;
    constexpr int k0 = T::stages[S].op_begin, k1 = T::stages[S].op_end;
    const bool active = w == T::LW || tid < (1u << w);
    uint32_t toff, roff[NA];
    stage_offsets<R>(&T::stages[S], w, tid, toff, roff);
    float2 a[NA], l[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        a[i] = active ? lds_ref(lds_psi, toff ^ roff[i]) : float2{0.f, 0.f};
        l[i] = active ? lds_ref(lds_lam, toff ^ roff[i]) : float2{0.f, 0.f};
    }
    static_for<0, k1 - k0>([&](auto J) __attribute__((always_inline)) {
        constexpr int K = k1 - 1 - std::decay_t<decltype(J)>::value;
        if constexpr (T::ops[K].grad_slot >= 0 && T::ops[K].kind == OP_DREG) {
            // a register diagonal folded from parameterised RZ rotations: one
            // partial per member slot (slots grad_slot + m in slot order)
            constexpr uint32_t mask = (uint32_t)T::ops[K].a;
            double vm[R];
            if constexpr (__builtin_popcount(mask) >= 2) grad_z_members<R>(a, l, mask, vm);
            static_for<0, R>([&](auto J) __attribute__((always_inline)) {
                constexpr int j = std::decay_t<decltype(J)>::value;
                if constexpr ((mask >> j) & 1u) {
                    constexpr int m = __builtin_popcount(mask & ((1u << j) - 1u));
                    double v;
                    if constexpr (__builtin_popcount(mask) >= 2) v = vm[j];
                    else v = wave_sum(grad_z_reg<R, j>(a, l));
                    if ((tid & 63) == 0) gpart[(int64_t)(T::ops[K].grad_slot + m) * slot_stride + part_index] = v;
                }
            });
        } else if constexpr (T::ops[K].grad_slot >= 0) {
            const double v = wave_sum(spec_grad<T, K>(a, l, tid, base));
            if ((tid & 63) == 0) gpart[(int64_t)T::ops[K].grad_slot * slot_stride + part_index] = v;
        }
        spec_op<T, K, true>(dpool, tid, base, a, l);
    });
    if (active) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            lds_ref(lds_psi, toff ^ roff[i]) = a[i];
            lds_ref(lds_lam, toff ^ roff[i]) = l[i];
        }
    }
    __syncthreads();
}

// One partition of the adjoint walk, as reverse_kernel: the checkpointed psi
// and lambda tiles into LDS, the stages last to first, lambda back to HBM.
template <class T>
__device__ __forceinline__ void spec_reverse(const float2 *__restrict__ psi_src, float2 *__restrict__ lam,
                                             const float *__restrict__ dpool, double *__restrict__ gpart,
                                             int64_t slot_stride)
{
    extern __shared__ float2 lds[];
    const DevPart *__restrict__ P = &T::part;
    const uint32_t tid = threadIdx.x;
    float2 *lds_psi = lds, *lds_lam = lds + (1u << T::part.t);
    const uint64_t base = tile_base<T::R, T::LW>(P, xcd_tile(blockIdx.x, gridDim.x, P));
    load_pairs<T::LW>(psi_src, lds_psi, P, base, tid);
    load_pairs<T::LW>(lam, lds_lam, P, base, tid);
    __syncthreads();
    constexpr int waves = (1 << T::LW) >= 64 ? (1 << T::LW) / 64 : 1;
    const int64_t part_index = (int64_t)blockIdx.x * waves + (tid >> 6);
    constexpr int ns = T::part.stage_end - T::part.stage_begin;
    static_for<0, ns>([&](auto J) __attribute__((always_inline)) {
        spec_reverse_stage<T, T::part.stage_end - 1 - std::decay_t<decltype(J)>::value>(lds_psi, lds_lam, dpool, gpart,
                                                                                       slot_stride, part_index, tid,
                                                                                       base);
    });
    store_pairs<T::LW>(lam, lds_lam, P, base, tid);
}

// Batched plans: the circuits of one structure share a table type T (the
// structure's one partition covers the whole state, so T::part.t = n).  The
// forward walk of such a circuit on its LDS tile, ending with a barrier.
template <class T, int S0, int S1>
__device__ __noinline__ void spec_bchunk(float2 *lds, const float *__restrict__ cpool, uint32_t tid)
{
    static_for<S0, S1>([&](auto S) __attribute__((always_inline)) {
        // a fresh copy of tid per stage: with 1024 threads a lane has 128
        // registers, too few to keep every stage's addresses computed ahead
        uint32_t t = tid;
        asm volatile("" : "+v"(t));
        spec_stage<T, std::decay_t<decltype(S)>::value>(lds, cpool, t, 0);
    });
}

// Stages in chunks of BCHUNK, each chunk a function of its own: the compile
// time of one long straight-line function grows faster than its length.
constexpr int BCHUNK = 4;

template <class T>
__device__ __forceinline__ void spec_bforward(float2 *lds, const float *__restrict__ cpool, uint32_t tid)
{
    constexpr int s0 = T::part.stage_begin, s1 = T::part.stage_end;
    static_for<0, (s1 - s0 + BCHUNK - 1) / BCHUNK>([&](auto C) __attribute__((always_inline)) {
        constexpr int a = s0 + BCHUNK * std::decay_t<decltype(C)>::value;
        constexpr int b = a + BCHUNK < s1 ? a + BCHUNK : s1;
        spec_bchunk<T, a, b>(lds, cpool, tid);
    });
}

}  // namespace qsv
