// Register-level gate application for the sweep kernels (gfx950, wave64).
//
// Each thread holds NA = 2^R amplitudes of a tile in registers.  Bit j of the
// register index is the tile qubit in register slot j; the other tile qubits
// are thread-id bits (lanes and waves); qubits outside the tile are bits of
// the tile index.  A gate whose qubits that must be local (Section 4.2) are
// register slots is applied entirely in registers; diagonal factors and
// controls may sit anywhere and are evaluated per amplitude from a 32-bit
// pattern: bit i of the pattern is the qubit's value for register index i.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "plan.h"

namespace qsv {

template <int J>
using IC = std::integral_constant<int, J>;

// Call f(IC<j>) for a runtime register slot j < R.
template <int R, typename F>
__device__ __forceinline__ void on_reg(int j, F &&f)
{
    switch (j) {
    case 0: f(IC<0>{}); break;
    case 1: if constexpr (R > 1) f(IC<1>{}); break;
    case 2: if constexpr (R > 2) f(IC<2>{}); break;
    case 3: if constexpr (R > 3) f(IC<3>{}); break;
    case 4: if constexpr (R > 4) f(IC<4>{}); break;
    default: break;
    }
}

__device__ __forceinline__ uint32_t reg_pattern(int j)
{
    switch (j) {
    case 0: return 0xAAAAAAAAu;
    case 1: return 0xCCCCCCCCu;
    case 2: return 0xF0F0F0F0u;
    case 3: return 0xFF00FF00u;
    default: return 0xFFFF0000u;
    }
}

// Pattern of a qubit location for this thread and tile.
__device__ __forceinline__ uint32_t loc_pattern(int32_t loc, uint32_t tid, uint64_t base)
{
    const int k = loc & 0x3F;
    switch (loc & LOC_MASK) {
    case LOC_REG: return reg_pattern(k);
    case LOC_THR: return ((tid >> k) & 1u) ? 0xFFFFFFFFu : 0u;
    default: return ((base >> k) & 1ull) ? 0xFFFFFFFFu : 0u;
    }
}

struct C2 {
    float r, i;
};

// The 8 floats of a 2x2 gate matrix (or 4 diagonal entries), loaded as one
// scalar block so the next op's matrix can be fetched while this one runs.
struct M8 {
    float v[8];
};

__device__ __forceinline__ M8 load_m8(const float *__restrict__ pool, int32_t mat)
{
    return *reinterpret_cast<const M8 *>(pool + (mat < 0 ? 0 : mat));
}

__device__ __forceinline__ C2 ld2(const float *__restrict__ m, int k, bool conj)
{
    return C2{m[2 * k], conj ? -m[2 * k + 1] : m[2 * k + 1]};
}

// a <- u0 x + u1 y (complex)
__device__ __forceinline__ float2 cmac2(C2 u0, float2 x, C2 u1, float2 y)
{
    float2 o;
    o.x = u0.r * x.x - u0.i * x.y + u1.r * y.x - u1.i * y.y;
    o.y = u0.r * x.y + u0.i * x.x + u1.r * y.y + u1.i * y.x;
    return o;
}

__device__ __forceinline__ float2 cmul(float2 a, C2 d)
{
    return float2{a.x * d.r - a.y * d.i, a.x * d.i + a.y * d.r};
}

// ---------------------------------------------------------------------------
// Dense 2x2 on register slot J.  DAG applies the conjugate transpose.
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_u1(float2 (&a)[1 << R], const float *__restrict__ m)
{
    C2 m00 = ld2(m, 0, DAG), m01 = ld2(m, DAG ? 2 : 1, DAG), m10 = ld2(m, DAG ? 1 : 2, DAG), m11 = ld2(m, 3, DAG);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        float2 x = a[i], y = a[i | (1 << J)];
        a[i] = cmac2(m00, x, m01, y);
        a[i | (1 << J)] = cmac2(m10, x, m11, y);
    }
}

// Real 2x2 on register slot J (real parts of the stored matrix).
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_r1(float2 (&a)[1 << R], const float *__restrict__ m)
{
    float m00 = m[0], m01 = m[DAG ? 4 : 2], m10 = m[DAG ? 2 : 4], m11 = m[6];
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        float2 x = a[i], y = a[i | (1 << J)];
        a[i] = float2{m00 * x.x + m01 * y.x, m00 * x.y + m01 * y.y};
        a[i | (1 << J)] = float2{m10 * x.x + m11 * y.x, m10 * x.y + m11 * y.y};
    }
}

// Diagonal 2x2 on a qubit anywhere (pattern p).
template <int R, bool DAG>
__device__ __forceinline__ void g_d1(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t p)
{
    C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 3, DAG);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        bool s = (p >> i) & 1u;
        a[i] = cmul(a[i], C2{s ? d1.r : d0.r, s ? d1.i : d0.i});
    }
}

// Diagonal over the register index: a[i] *= d[i] (d uniform across threads).
template <int R, bool DAG>
__device__ __forceinline__ void g_dreg(float2 (&a)[1 << R], const float *__restrict__ d)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) a[i] = cmul(a[i], C2{d[2 * i], DAG ? -d[2 * i + 1] : d[2 * i + 1]});
}

// -1 where both qubits are 1 (pattern p = pa & pb).
template <int R>
__device__ __forceinline__ void g_cz(float2 (&a)[1 << R], uint32_t p)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if ((p >> i) & 1u) a[i] = float2{-a[i].x, -a[i].y};
    }
}

// Diagonal 4x4 on two qubits anywhere: entry j = bit(a) + 2 bit(b).
template <int R, bool DAG>
__device__ __forceinline__ void g_d2(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t pa, uint32_t pb)
{
    C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 1, DAG), d2 = ld2(m, 2, DAG), d3 = ld2(m, 3, DAG);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        bool sa = (pa >> i) & 1u, sb = (pb >> i) & 1u;
        C2 lo{sa ? d1.r : d0.r, sa ? d1.i : d0.i};
        C2 hi{sa ? d3.r : d2.r, sa ? d3.i : d2.i};
        a[i] = cmul(a[i], C2{sb ? hi.r : lo.r, sb ? hi.i : lo.i});
    }
}

// X on register slot J where the control pattern pc is 1.
template <int R, int J>
__device__ __forceinline__ void g_cx(float2 (&a)[1 << R], uint32_t pc)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        bool s = (pc >> i) & 1u;
        float2 x = a[i], y = a[i | (1 << J)];
        a[i] = s ? y : x;
        a[i | (1 << J)] = s ? x : y;
    }
}

// General 2x2 on register slot J where the control pattern pc is 1.
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_cu(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t pc)
{
    C2 m00 = ld2(m, 0, DAG), m01 = ld2(m, DAG ? 2 : 1, DAG), m10 = ld2(m, DAG ? 1 : 2, DAG), m11 = ld2(m, 3, DAG);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        bool s = (pc >> i) & 1u;
        float2 x = a[i], y = a[i | (1 << J)];
        float2 nx = cmac2(m00, x, m01, y), ny = cmac2(m10, x, m11, y);
        a[i] = s ? nx : x;
        a[i | (1 << J)] = s ? ny : y;
    }
}

// Dense 4x4 on register slots (JA, JB); local index j = b(JA) + 2 b(JB).
template <int R, int JA, int JB, bool DAG>
__device__ __forceinline__ void g_u2(float2 (&a)[1 << R], const float *__restrict__ m)
{
    // row r, column c of U (or of U^dagger)
    auto U = [&](int r, int c) __attribute__((always_inline)) { return DAG ? ld2(m, c * 4 + r, true) : ld2(m, r * 4 + c, false); };
    const C2 u00 = U(0, 0), u01 = U(0, 1), u02 = U(0, 2), u03 = U(0, 3);
    const C2 u10 = U(1, 0), u11 = U(1, 1), u12 = U(1, 2), u13 = U(1, 3);
    const C2 u20 = U(2, 0), u21 = U(2, 1), u22 = U(2, 2), u23 = U(2, 3);
    const C2 u30 = U(3, 0), u31 = U(3, 1), u32 = U(3, 2), u33 = U(3, 3);
    constexpr int A = 1 << JA, B = 1 << JB;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (A | B)) continue;
        const float2 v0 = a[i], v1 = a[i | A], v2 = a[i | B], v3 = a[i | A | B];
        float2 o, p;
        o = cmac2(u00, v0, u01, v1); p = cmac2(u02, v2, u03, v3); a[i] = float2{o.x + p.x, o.y + p.y};
        o = cmac2(u10, v0, u11, v1); p = cmac2(u12, v2, u13, v3); a[i | A] = float2{o.x + p.x, o.y + p.y};
        o = cmac2(u20, v0, u21, v1); p = cmac2(u22, v2, u23, v3); a[i | B] = float2{o.x + p.x, o.y + p.y};
        o = cmac2(u30, v0, u31, v1); p = cmac2(u32, v2, u33, v3); a[i | A | B] = float2{o.x + p.x, o.y + p.y};
    }
}

template <int R, int JA, int JB>
__device__ __forceinline__ void g_swap(float2 (&a)[1 << R])
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & ((1 << JA) | (1 << JB))) continue;
        float2 t = a[i | (1 << JA)];
        a[i | (1 << JA)] = a[i | (1 << JB)];
        a[i | (1 << JB)] = t;
    }
}

// Apply one op (or its conjugate transpose) to a thread's amplitudes.
// mm holds the op's 8 leading matrix floats (load_m8); dense 4x4 ops read the
// rest from the pool.
template <int R, bool DAG>
__device__ __forceinline__ void apply_op(float2 (&a)[1 << R], const DevOp &o, const M8 &mm,
                                         const float *__restrict__ pool, uint32_t tid, uint64_t base)
{
    const float *m = mm.v;
    const float *__restrict__ m32 = pool + (o.mat < 0 ? 0 : o.mat);
    switch (o.kind) {
    case OP_U1: on_reg<R>(o.a & 0x3F, [&](auto J) __attribute__((always_inline)) { g_u1<R, std::decay_t<decltype(J)>::value, DAG>(a, m); }); break;
    case OP_R1: on_reg<R>(o.a & 0x3F, [&](auto J) __attribute__((always_inline)) { g_r1<R, std::decay_t<decltype(J)>::value, DAG>(a, m); }); break;
    case OP_D1: g_d1<R, DAG>(a, m, loc_pattern(o.a, tid, base)); break;
    case OP_DREG: g_dreg<R, DAG>(a, m32); break;
    case OP_CZ: g_cz<R>(a, loc_pattern(o.a, tid, base) & loc_pattern(o.b, tid, base)); break;
    case OP_D2: g_d2<R, DAG>(a, m, loc_pattern(o.a, tid, base), loc_pattern(o.b, tid, base)); break;
    case OP_CX: {
        uint32_t pc = loc_pattern(o.a, tid, base);
        on_reg<R>(o.b & 0x3F, [&](auto J) __attribute__((always_inline)) { g_cx<R, std::decay_t<decltype(J)>::value>(a, pc); });
        break;
    }
    case OP_CU: {
        uint32_t pc = loc_pattern(o.a, tid, base);
        on_reg<R>(o.b & 0x3F, [&](auto J) __attribute__((always_inline)) { g_cu<R, std::decay_t<decltype(J)>::value, DAG>(a, m, pc); });
        break;
    }
    case OP_U2:
        if constexpr (R >= 2) {
            on_reg<R>(o.a & 0x3F, [&](auto JA) __attribute__((always_inline)) {
                on_reg<R>(o.b & 0x3F, [&](auto JB) __attribute__((always_inline)) {
                    if constexpr (std::decay_t<decltype(JA)>::value != std::decay_t<decltype(JB)>::value)
                        g_u2<R, std::decay_t<decltype(JA)>::value, std::decay_t<decltype(JB)>::value, DAG>(a, m32);
                });
            });
        }
        break;
    case OP_SWAP:
        if constexpr (R >= 2) {
            on_reg<R>(o.a & 0x3F, [&](auto JA) __attribute__((always_inline)) {
                on_reg<R>(o.b & 0x3F, [&](auto JB) __attribute__((always_inline)) {
                    if constexpr (std::decay_t<decltype(JA)>::value != std::decay_t<decltype(JB)>::value)
                        g_swap<R, std::decay_t<decltype(JA)>::value, std::decay_t<decltype(JB)>::value>(a);
                });
            });
        }
        break;
    default: break;
    }
}

template <int R, bool DAG>
__device__ __forceinline__ void apply_op(float2 (&a)[1 << R], const DevOp &o, const float *__restrict__ pool,
                                         uint32_t tid, uint64_t base)
{
    apply_op<R, DAG>(a, o, load_m8(pool, o.mat), pool, tid, base);
}

// ---------------------------------------------------------------------------
// Adjoint helpers: Im <lambda|P|psi> for the generator P of a rotation
// exp(-i a P / 2), over one thread's amplitudes, in float64.
__device__ __forceinline__ double im_conj_mul(float2 l, float2 a) { return (double)l.x * a.y - (double)l.y * a.x; }
__device__ __forceinline__ double re_conj_mul(float2 l, float2 a) { return (double)l.x * a.x + (double)l.y * a.y; }

template <int R, int J>
__device__ __forceinline__ double grad_pairs(const float2 (&a)[1 << R], const float2 (&l)[1 << R], bool y_gen)
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        const float2 a0 = a[i], a1 = a[i | (1 << J)], l0 = l[i], l1 = l[i | (1 << J)];
        if (y_gen)  // Y: (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0
            acc += re_conj_mul(l1, a0) - re_conj_mul(l0, a1);
        else        // X: (X psi)_0 = psi_1, (X psi)_1 = psi_0
            acc += im_conj_mul(l0, a1) + im_conj_mul(l1, a0);
    }
    return acc;
}

// Im <lambda|P|psi> over this thread's amplitudes for the op's generator.
template <int R>
__device__ __forceinline__ double grad_term(const float2 (&a)[1 << R], const float2 (&l)[1 << R], const DevOp &o,
                                            uint32_t tid, uint64_t base)
{
    double acc = 0.0;
    if (o.gen == GEN_Z || o.gen == GEN_ZZ) {
        uint32_t p = loc_pattern(o.a, tid, base);
        if (o.gen == GEN_ZZ) p ^= loc_pattern(o.b, tid, base);
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) {
            const double v = im_conj_mul(l[i], a[i]);
            acc += ((p >> i) & 1u) ? -v : v;
        }
    } else {
        const bool y = o.gen == GEN_Y;
        on_reg<R>(o.a & 0x3F, [&](auto J) __attribute__((always_inline)) { acc = grad_pairs<R, std::decay_t<decltype(J)>::value>(a, l, y); });
    }
    return acc;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// XOR swizzle of an 8-byte LDS slot: bits 5-9 and 10-14 of the tile position
// are folded into bits 0-4, so 32 lanes whose positions differ in bits with
// distinct residues mod 5 hit distinct bank pairs.  swz is linear over GF(2):
// for positions with disjoint bits swz(a | b) = swz(a) ^ swz(b), so a thread
// swizzles its thread-bit offset once and the register-bit offsets (uniform)
// are swizzled in scalar registers.
__device__ __forceinline__ uint32_t swz(uint32_t c) { return c ^ ((c >> 5) & 31u) ^ ((c >> 10) & 31u); }

// Swizzled LDS offsets of a stage layout: the thread's own part and the
// register-index parts (uniform).
template <int R>
__device__ __forceinline__ void stage_offsets(const DevStage *__restrict__ S, int w, uint32_t tid, uint32_t &toff,
                                              uint32_t (&roff)[1 << R])
{
    uint32_t t = 0;
    for (int b = 0; b < w; ++b) t |= ((tid >> b) & 1u) << S->thrpos[b];
    toff = swz(t);
    uint32_t r[1 << R];
    r[0] = 0;
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) r[i] = r[i & (i - 1)] | (1u << S->regpos[__builtin_ctz(i)]);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) roff[i] = swz(r[i]);
}

// Run the register stages [s0, s1) of a tile held in LDS.
template <int R, bool DAG>
__device__ __forceinline__ void run_stages(float2 *lds, const DevStage *__restrict__ stages, const DevOp *__restrict__ ops,
                                           const float *__restrict__ pool, int s0, int s1, int w, uint32_t tid,
                                           uint64_t base)
{
    constexpr int NA = 1 << R;
    const bool active = tid < (1u << w);
    for (int s = s0; s < s1; ++s) {
        const DevStage *__restrict__ S = stages + s;
        if (active) {
            uint32_t toff, roff[NA];
            stage_offsets<R>(S, w, tid, toff, roff);
            float2 a[NA];
#pragma unroll
            for (int i = 0; i < NA; ++i) a[i] = lds[toff ^ roff[i]];
            const int k0 = S->op_begin, k1 = S->op_end;
            if (k0 < k1) {  // the next op and its matrix are fetched while the current one runs
                DevOp cur = ops[k0];
                M8 mc = load_m8(pool, cur.mat);
                for (int k = k0; k < k1; ++k) {
                    const int kn = k + 1 < k1 ? k + 1 : k;
                    const DevOp nxt = ops[kn];
                    const M8 mn = load_m8(pool, nxt.mat);
                    apply_op<R, DAG>(a, cur, mc, pool, tid, base);
                    cur = nxt;
                    mc = mn;
                }
            }
            asm volatile("" : "+v"(toff));  // recompute the write-back addresses instead of keeping 2^R live
#pragma unroll
            for (int i = 0; i < NA; ++i) lds[toff ^ roff[i]] = a[i];
        }
        __syncthreads();
    }
}

}  // namespace qsv
