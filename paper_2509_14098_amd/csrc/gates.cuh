// Register-level gate application for the sweep kernels (gfx950, wave64).
//
// Each thread holds NA = 2^R amplitudes of a tile in registers.  Bit j of the
// register index is the tile qubit in register slot j; the other tile qubits
// are thread-id bits (lanes and waves); qubits outside the tile are bits of
// the tile index.  A gate whose qubits that must be local (Section 4.2) are
// register slots is applied entirely in registers; diagonal factors and
// controls may sit anywhere: on a register slot they select amplitudes by
// register index, on a thread or tile-index qubit they are one value per
// thread.  Every gate body updates the amplitudes in place (see fma_ip).
//
// The in-place bodies have two forms of the same arithmetic: gfx950
// instructions with tied registers (QSV_INPLACE_ASM, for the table-driven
// kernels) and plain C++, used by the specialised kernels and when the test
// emulator compiles this header for the host.
#pragma once
#ifndef __HIPCC_RTC__  // hipRTC provides the runtime declarations itself
#include <hip/hip_runtime.h>
#endif

#include <type_traits>

#include "plan.h"

namespace qsv {

template <int J>
using IC = std::integral_constant<int, J>;

// A uniform value whose derivation the compiler cannot see.  Op dispatch tests
// single bits of such values, so each op body becomes a two-way branch that
// the amplitudes pass through unchanged when skipped; a multi-way switch
// instead gives every case its own register assignment and costs register
// copies wherever the cases merge.
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    v = __builtin_amdgcn_readfirstlane(v);  // op fields are uniform; this states it where the compiler cannot prove it
    asm("" : "+s"(v));
#endif
    return v;
}

// Call f(IC<J>) for the register slot J whose bit is set in the one-hot
// (opaque) mask bits.
template <int R, typename F, int J = 0>
__device__ __forceinline__ void on_slot(uint32_t bits, F &&f)
{
    if constexpr (J < R) {
        if (bits & (1u << J)) f(IC<J>{});
        on_slot<R, F, J + 1>(bits, static_cast<F &&>(f));
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

// Value (0 or 1) of a thread or tile-index qubit for this thread and tile.
__device__ __forceinline__ uint32_t lane_bit(int32_t loc, uint32_t tid, uint64_t base)
{
    const int k = loc & 0x3F;
    return (loc & LOC_MASK) == LOC_THR ? (tid >> k) & 1u : (uint32_t)(base >> k) & 1u;
}

// The 8 floats of a 2x2 gate matrix (or 4 diagonal entries), loaded as one
// scalar block.
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

// The in-place instruction forms below are used in the table-driven kernels.
// Specialised kernels (straight-line code, no dispatch merges) define
// QSV_PLAIN_ARITH and get the plain expressions, which the compiler schedules
// and contracts freely.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(QSV_PLAIN_ARITH)
#define QSV_INPLACE_ASM 1
#else
#define QSV_INPLACE_ASM 0
#endif

// In-place updates x <- s x + t and x <- s x - t with s uniform.  Written as
// instructions whose result is tied to x's register so that an op's outputs
// stay in the registers its inputs came from: the op dispatch loop then needs
// no register copies where its cases merge.  (The test emulator compiles the
// same expressions for the host.)
__device__ __forceinline__ void fma_ip(float &x, float s, float t)
{
#if QSV_INPLACE_ASM
    asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x) : "s"(s), "v"(t));
#else
    x = s * x + t;
#endif
}
__device__ __forceinline__ void fms_ip(float &x, float s, float t)
{
#if QSV_INPLACE_ASM
    asm("v_fma_f32 %0, %1, %0, -%2" : "+v"(x) : "s"(s), "v"(t));
#else
    x = s * x - t;
#endif
}

// x <- s x + t with s per lane
__device__ __forceinline__ void fma_ipv(float &x, float s, float t)
{
#if QSV_INPLACE_ASM
    asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x) : "v"(s), "v"(t));
#else
    x = s * x + t;
#endif
}
__device__ __forceinline__ void fms_ipv(float &x, float s, float t)
{
#if QSV_INPLACE_ASM
    asm("v_fma_f32 %0, %1, %0, -%2" : "+v"(x) : "v"(s), "v"(t));
#else
    x = s * x - t;
#endif
}
// exchange two registers
__device__ __forceinline__ void swap_ip(float &x, float &y)
{
#if QSV_INPLACE_ASM
    asm("v_swap_b32 %0, %1" : "+v"(x), "+v"(y));
#else
    const float t = x;
    x = y;
    y = t;
#endif
}
// x <- x + s y with s uniform, in place
__device__ __forceinline__ void fmac_ip(float &x, float s, float y)
{
#if QSV_INPLACE_ASM
    asm("v_fmac_f32 %0, %1, %2" : "+v"(x) : "s"(s), "v"(y));
#else
    x = s * y + x;
#endif
}

// x <- x ^ d (bit pattern), in place
__device__ __forceinline__ void xor_ip(float &x, uint32_t d)
{
#if QSV_INPLACE_ASM
    asm("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(d));
#else
    x = __uint_as_float(__float_as_uint(x) ^ d);
#endif
}
// x <- x ^ d with d uniform
__device__ __forceinline__ void xor_ips(float &x, uint32_t d)
{
#if QSV_INPLACE_ASM
    asm("v_xor_b32 %0, %1, %0" : "+v"(x) : "s"(d));
#else
    x = __uint_as_float(__float_as_uint(x) ^ d);
#endif
}

// a <- a d (complex, d per lane), in place
__device__ __forceinline__ void cmul_ipv(float2 &a, float dr, float di)
{
    const float t = a.y * di, u = a.x * di;
    fms_ipv(a.x, dr, t);
    fma_ipv(a.y, dr, u);
}

// a <- a d (complex, d uniform), in place
__device__ __forceinline__ void cmul_ip(float2 &a, float dr, float di)
{
    const float t = a.y * di, u = a.x * di;
    fms_ip(a.x, dr, t);
    fma_ip(a.y, dr, u);
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
        float2 &x = a[i], &y = a[i | (1 << J)];
        // every term but the diagonal one first, then the diagonal term in place
        const float t0 = m01.r * y.x - m00.i * x.y - m01.i * y.y;
        const float t1 = m01.r * y.y + m00.i * x.x + m01.i * y.x;
        const float t2 = m10.r * x.x - m10.i * x.y - m11.i * y.y;
        const float t3 = m10.r * x.y + m10.i * x.x + m11.i * y.x;
        fma_ip(x.x, m00.r, t0);
        fma_ip(x.y, m00.r, t1);
        fma_ip(y.x, m11.r, t2);
        fma_ip(y.y, m11.r, t3);
    }
}

// Real 2x2 on register slot J (real parts of the stored matrix).
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_r1(float2 (&a)[1 << R], const float *__restrict__ m)
{
    const float m00 = m[0], m01 = m[DAG ? 4 : 2], m10 = m[DAG ? 2 : 4], m11 = m[6];
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        float2 &x = a[i], &y = a[i | (1 << J)];
        const float tx = m01 * y.x, ty = m01 * y.y, ux = m10 * x.x, uy = m10 * x.y;
        fma_ip(x.x, m00, tx);
        fma_ip(x.y, m00, ty);
        fma_ip(y.x, m11, ux);
        fma_ip(y.y, m11, uy);
    }
}

// Diagonal 2x2 on register slot J.
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_d1(float2 (&a)[1 << R], const float *__restrict__ m)
{
    const C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 3, DAG);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        const C2 d = (i >> J) & 1 ? d1 : d0;
        cmul_ip(a[i], d.r, d.i);
    }
}

// Diagonal 2x2 on a thread or tile-index qubit whose value here is bit: one
// factor for all of this thread's amplitudes.
template <int R, bool DAG>
__device__ __forceinline__ void g_d1_lane(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t bit)
{
    const C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 3, DAG);
    const float dr = bit ? d1.r : d0.r, di = bit ? d1.i : d0.i;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) cmul_ipv(a[i], dr, di);
}

// Rotation [[c, -s], [s, c]] with c >= 0 on register slot J as three shears
// (x += t y; y += s x; x += t y with t = -s / (1 + c)): three in-place
// multiply-adds per pair component, |t| <= 1.  The conjugate transpose is the
// rotation by the opposite angle: (t, s) -> (-t, -s).
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_rot(float2 (&a)[1 << R], float t, float sn)
{
    if (DAG) {
        t = -t;
        sn = -sn;
    }
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        float2 &x = a[i], &y = a[i | (1 << J)];
        fmac_ip(x.x, t, y.x);
        fmac_ip(x.y, t, y.y);
        fmac_ip(y.x, sn, x.x);
        fmac_ip(y.y, sn, x.y);
        fmac_ip(x.x, t, y.x);
        fmac_ip(x.y, t, y.y);
    }
}

// Rotations on the register slots in mask (slot J's (t, s) at r + 2 J).
template <int R, bool DAG, int J = 0>
__device__ __forceinline__ void g_rot_layer(float2 (&a)[1 << R], const float *__restrict__ r, uint32_t mask)
{
    if constexpr (J < R) {
        if ((mask >> J) & 1u) g_rot<R, J, DAG>(a, r[2 * J], r[2 * J + 1]);
        g_rot_layer<R, DAG, J + 1>(a, r, mask);
    }
}

// Diagonal over the register index: a[i] *= d[i] (d uniform across threads).
template <int R, bool DAG>
__device__ __forceinline__ void g_dreg(float2 (&a)[1 << R], const float *__restrict__ d)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) cmul_ip(a[i], d[2 * i], DAG ? -d[2 * i + 1] : d[2 * i + 1]);
}

// Layer op: register diagonal then rotations (the conjugate transpose reverses
// the order).  Straight-line code, so consecutive layers run without the
// register copies a multi-way dispatch costs.
template <int R, bool DAG>
__device__ __forceinline__ void g_layer(float2 (&a)[1 << R], const float *__restrict__ p, uint32_t mask)
{
    if (!DAG) g_dreg<R, false>(a, p);
    g_rot_layer<R, DAG>(a, p + 2 * (1 << R), mask);
    if (DAG) g_dreg<R, true>(a, p);
}

// CZ as sign-bit flips.  Both qubits in register slots: the uniform pattern p
// (bit i set where both are 1).
template <int R>
__device__ __forceinline__ void g_cz(float2 (&a)[1 << R], uint32_t p)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        const uint32_t sg = ((p >> i) & 1u) << 31;
        xor_ips(a[i].x, sg);
        xor_ips(a[i].y, sg);
    }
}

// Register slot J and a thread or tile-index qubit (sign bit sg: that qubit's value << 31).
template <int R, int J>
__device__ __forceinline__ void g_cz_rt(float2 (&a)[1 << R], uint32_t sg)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (!((i >> J) & 1)) continue;
        xor_ip(a[i].x, sg);
        xor_ip(a[i].y, sg);
    }
}

// Two thread or tile-index qubits: one sign for all of this thread's amplitudes.
template <int R>
__device__ __forceinline__ void g_cz_tt(float2 (&a)[1 << R], uint32_t sg)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        xor_ip(a[i].x, sg);
        xor_ip(a[i].y, sg);
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
        cmul_ipv(a[i], sb ? hi.r : lo.r, sb ? hi.i : lo.i);
    }
}

// Diagonal 4x4 on register slot J (a) and a thread or tile-index qubit (b)
// whose value here is bit: two factors per thread, picked by the slot's bit.
template <int R, int J, bool DAG>
__device__ __forceinline__ void g_d2_rt(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t bit, bool lo_one)
{
    const C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 1, DAG), d2 = ld2(m, 2, DAG), d3 = ld2(m, 3, DAG);
    const float hr = bit ? d3.r : d1.r, hi = bit ? d3.i : d1.i;  // slot bit 1
#pragma unroll
    for (int i = 0; i < (1 << R); ++i)
        if ((i >> J) & 1) cmul_ipv(a[i], hr, hi);
    if (!lo_one) {  // slot bit 0 (skipped for controlled phases, whose factors there are 1)
        const float lr = bit ? d2.r : d0.r, li = bit ? d2.i : d0.i;
#pragma unroll
        for (int i = 0; i < (1 << R); ++i)
            if (!((i >> J) & 1)) cmul_ipv(a[i], lr, li);
    }
}

// Diagonal 4x4 on two thread or tile-index qubits: one factor per thread.
template <int R, bool DAG>
__device__ __forceinline__ void g_d2_tt(float2 (&a)[1 << R], const float *__restrict__ m, uint32_t j)
{
    const C2 d0 = ld2(m, 0, DAG), d1 = ld2(m, 1, DAG), d2 = ld2(m, 2, DAG), d3 = ld2(m, 3, DAG);
    const float r = j == 0 ? d0.r : j == 1 ? d1.r : j == 2 ? d2.r : d3.r;
    const float im = j == 0 ? d0.i : j == 1 ? d1.i : j == 2 ? d2.i : d3.i;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) cmul_ipv(a[i], r, im);
}

// X on register slot J controlled by register slot C: a fixed permutation.
template <int R, int C, int J>
__device__ __forceinline__ void g_cx_reg(float2 (&a)[1 << R])
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if ((i & (1 << J)) || !(i & (1 << C))) continue;
        swap_ip(a[i].x, a[i | (1 << J)].x);
        swap_ip(a[i].y, a[i | (1 << J)].y);
    }
}

// X on register slot J where the thread's control bit is 1 (mask m: all ones or zero).
template <int R, int J>
__device__ __forceinline__ void g_cx_lane(float2 (&a)[1 << R], uint32_t m)
{
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        float2 &x = a[i], &y = a[i | (1 << J)];
        const uint32_t dr = (__float_as_uint(x.x) ^ __float_as_uint(y.x)) & m;
        const uint32_t di = (__float_as_uint(x.y) ^ __float_as_uint(y.y)) & m;
        xor_ip(x.x, dr);
        xor_ip(y.x, dr);
        xor_ip(x.y, di);
        xor_ip(y.y, di);
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
        swap_ip(a[i | (1 << JA)].x, a[i | (1 << JB)].x);
        swap_ip(a[i | (1 << JA)].y, a[i | (1 << JB)].y);
    }
}

// After each array of a multi-array op when SEQ holds: the compiler may not
// interleave the arrays' updates (with 1024 threads a lane has 128 VGPRs, too
// few for psi and lambda to be updated together).
template <bool SEQ>
__device__ __forceinline__ void array_fence()
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (SEQ) __builtin_amdgcn_sched_barrier(0);
#endif
}

// Apply one op (or its conjugate transpose) to one or more amplitude arrays of
// a thread (the adjoint walk applies each op to psi and lambda in one pass:
// one dispatch; with SEQ one array after the other).  The op kind and the
// register slots are tested bit by bit on opaque one-hot masks (see opaque()).
template <int R, bool DAG, bool SEQ = false, typename... Arr>
__device__ __forceinline__ void apply_ops(const DevOp &o, const float *__restrict__ pool, uint32_t tid,
                                          uint64_t base, Arr &...as)
{
    constexpr bool F = SEQ && sizeof...(Arr) > 1;
    const float *__restrict__ m32 = pool + (o.mat < 0 ? 0 : o.mat);
    const uint32_t kb = opaque(1u << o.kind);
    const uint32_t ja = opaque(1u << (o.a & 0x3F)), jb = opaque(1u << (o.b & 0x3F));
#define QSV_J(x) std::decay_t<decltype(x)>::value
    if (kb & (1u << OP_LAYER)) ((g_layer<R, DAG>(as, m32, (uint32_t)o.a), array_fence<F>()), ...);
    if (kb & (1u << OP_DREG)) ((g_dreg<R, DAG>(as, m32), array_fence<F>()), ...);
    if (kb & (1u << OP_CZ_RT)) {
        const uint32_t sg = lane_bit(o.b, tid, base) << 31;
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { ((g_cz_rt<R, QSV_J(J)>(as, sg), array_fence<F>()), ...); });
    }
    if (kb & (1u << OP_CZ_TT)) {
        const uint32_t sg = (lane_bit(o.a, tid, base) & lane_bit(o.b, tid, base)) << 31;
        ((g_cz_tt<R>(as, sg), array_fence<F>()), ...);
    }
    if (kb & (1u << OP_CX)) {
        on_slot<R>(ja, [&](auto C) __attribute__((always_inline)) {
            on_slot<R>(jb, [&](auto J) __attribute__((always_inline)) {
                if constexpr (QSV_J(C) != QSV_J(J)) ((g_cx_reg<R, QSV_J(C), QSV_J(J)>(as), array_fence<F>()), ...);
            });
        });
    }
    if (kb & (1u << OP_CX_T)) {
        const uint32_t mk = 0u - lane_bit(o.a, tid, base);
        on_slot<R>(jb, [&](auto J) __attribute__((always_inline)) { ((g_cx_lane<R, QSV_J(J)>(as, mk), array_fence<F>()), ...); });
    }
    // the kinds that fused stages use least are tested only when one of them is present
    constexpr uint32_t RARE = (1u << OP_U1) | (1u << OP_R1) | (1u << OP_CZ) | (1u << OP_D1) | (1u << OP_D1_T) |
                              (1u << OP_D2) | (1u << OP_D2_RT) | (1u << OP_D2_TT) | (1u << OP_CU) | (1u << OP_U2) |
                              (1u << OP_SWAP);
    if (!(kb & RARE)) return;
    const M8 mm = load_m8(pool, o.mat);  // the 8 leading matrix floats, one scalar load
    const float *m = mm.v;
    if (kb & (1u << OP_U1))
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { ((g_u1<R, QSV_J(J), DAG>(as, m), array_fence<F>()), ...); });
    if (kb & (1u << OP_R1))
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { ((g_r1<R, QSV_J(J), DAG>(as, m), array_fence<F>()), ...); });
    if (kb & (1u << OP_CZ)) {
        const uint32_t p = reg_pattern(o.a & 0x3F) & reg_pattern(o.b & 0x3F);
        ((g_cz<R>(as, p), array_fence<F>()), ...);
    }
    if (kb & (1u << OP_D1))
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { ((g_d1<R, QSV_J(J), DAG>(as, m), array_fence<F>()), ...); });
    if (kb & (1u << OP_D1_T)) {
        const uint32_t bit = lane_bit(o.a, tid, base);
        ((g_d1_lane<R, DAG>(as, m, bit), array_fence<F>()), ...);
    }
    if (kb & (1u << OP_D2)) {
        const uint32_t pa = loc_pattern(o.a, tid, base), pb = loc_pattern(o.b, tid, base);
        ((g_d2<R, DAG>(as, m, pa, pb), array_fence<F>()), ...);
    }
    if (kb & (1u << OP_D2_RT)) {
        const uint32_t bit = lane_bit(o.b, tid, base);
        const bool lo_one = o.flags & 1;
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { ((g_d2_rt<R, QSV_J(J), DAG>(as, m, bit, lo_one), array_fence<F>()), ...); });
    }
    if (kb & (1u << OP_D2_TT)) {
        const uint32_t j = lane_bit(o.a, tid, base) + 2u * lane_bit(o.b, tid, base);
        ((g_d2_tt<R, DAG>(as, m, j), array_fence<F>()), ...);
    }
    if (kb & (1u << OP_CU)) {
        const uint32_t pc = loc_pattern(o.a, tid, base);
        on_slot<R>(jb, [&](auto J) __attribute__((always_inline)) { ((g_cu<R, QSV_J(J), DAG>(as, m, pc), array_fence<F>()), ...); });
    }
    if constexpr (R >= 2) {
        if (kb & (1u << OP_U2)) {
            on_slot<R>(ja, [&](auto JA) __attribute__((always_inline)) {
                on_slot<R>(jb, [&](auto JB) __attribute__((always_inline)) {
                    if constexpr (QSV_J(JA) != QSV_J(JB)) ((g_u2<R, QSV_J(JA), QSV_J(JB), DAG>(as, m32), array_fence<F>()), ...);
                });
            });
        }
        if (kb & (1u << OP_SWAP)) {
            on_slot<R>(ja, [&](auto JA) __attribute__((always_inline)) {
                on_slot<R>(jb, [&](auto JB) __attribute__((always_inline)) {
                    if constexpr (QSV_J(JA) != QSV_J(JB)) ((g_swap<R, QSV_J(JA), QSV_J(JB)>(as), array_fence<F>()), ...);
                });
            });
        }
    }
#undef QSV_J
}

template <int R, bool DAG>
__device__ __forceinline__ void apply_op(float2 (&a)[1 << R], const DevOp &o, const float *__restrict__ pool,
                                         uint32_t tid, uint64_t base)
{
    apply_ops<R, DAG>(o, pool, tid, base, a);
}

// The op's conjugate transpose on psi and lambda together (adjoint walk).
template <int R>
__device__ __forceinline__ void apply_op_dag2(float2 (&a)[1 << R], float2 (&l)[1 << R], const DevOp &o,
                                              const float *__restrict__ pool, uint32_t tid, uint64_t base)
{
    apply_ops<R, true>(o, pool, tid, base, a, l);
}

// ---------------------------------------------------------------------------
// Adjoint helpers: Im <lambda|P|psi> for the generator P of a rotation
// exp(-i a P / 2), over one thread's amplitudes: each amplitude's product in
// float32 (one multiply and one fused multiply-add, relative error 2^-23 of
// its terms, below the float32 state's own rounding), the sum in float64.
__device__ __forceinline__ double acc_im(double acc, float2 l, float2 a)
{
    return acc + (double)__builtin_fmaf(l.x, a.y, -(l.y * a.x));  // acc + Im(conj(l) a)
}
__device__ __forceinline__ double acc_re(double acc, float2 l, float2 a)
{
    return acc + (double)__builtin_fmaf(l.x, a.x, l.y * a.y);  // acc + Re(conj(l) a)
}

template <int R, int J, bool Y>
__device__ __forceinline__ double grad_pairs(const float2 (&a)[1 << R], const float2 (&l)[1 << R])
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (i & (1 << J)) continue;
        const float2 a0 = a[i], a1 = a[i | (1 << J)], l0 = l[i], l1 = l[i | (1 << J)];
        if (Y) {  // Y: (Y psi)_0 = -i psi_1, (Y psi)_1 = i psi_0
            acc = acc_re(acc, l1, a0);
            acc = acc_re(acc, float2{-l0.x, -l0.y}, a1);
        } else {  // X: (X psi)_0 = psi_1, (X psi)_1 = psi_0
            acc = acc_im(acc, l0, a1);
            acc = acc_im(acc, l1, a0);
        }
    }
    return acc;
}

// Z on register slot J: the sign of each term is fixed by the register index.
template <int R, int J>
__device__ __forceinline__ double grad_z_reg(const float2 (&a)[1 << R], const float2 (&l)[1 << R])
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        acc = acc_im(acc, ((i >> J) & 1) ? float2{-l[i].x, -l[i].y} : l[i], a[i]);
    }
    return acc;
}

// Im <lambda|P|psi> over this thread's amplitudes for the op's generator.
template <int R>
__device__ __forceinline__ double grad_term(const float2 (&a)[1 << R], const float2 (&l)[1 << R], const DevOp &o,
                                            uint32_t tid, uint64_t base)
{
    double acc = 0.0;
    const uint32_t ja = opaque(1u << (o.a & 0x3F));
    if (o.gen == GEN_Z && (o.a & LOC_MASK) == LOC_REG) {
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { acc = grad_z_reg<R, std::decay_t<decltype(J)>::value>(a, l); });
    } else if (o.gen == GEN_Z || o.gen == GEN_ZZ) {
        uint32_t p = loc_pattern(o.a, tid, base);
        if (o.gen == GEN_ZZ) p ^= loc_pattern(o.b, tid, base);
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) {
            acc = acc_im(acc, ((p >> i) & 1u) ? float2{-l[i].x, -l[i].y} : l[i], a[i]);
        }
    } else if (o.gen == GEN_Y) {
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { acc = grad_pairs<R, std::decay_t<decltype(J)>::value, true>(a, l); });
    } else {
        on_slot<R>(ja, [&](auto J) __attribute__((always_inline)) { acc = grad_pairs<R, std::decay_t<decltype(J)>::value, false>(a, l); });
    }
    return acc;
}

// Tile handled by workgroup b of nblk.  Workgroups are handed to the chip's 8
// XCDs round-robin (b mod 8) and each XCD has its own L2.  The 2^g tiles that
// differ only in global qubits below 4 (g = number of such qubits) share
// 128-byte lines of the state, so they are given to consecutive workgroups of
// one XCD: each line is then fetched from HBM once instead of once per XCD.
__device__ __forceinline__ uint64_t xcd_tile(uint32_t b, uint32_t nblk, const DevPart *__restrict__ P)
{
    int g = 0;
    while (g < P->n_glb && P->gq[g] < 4) ++g;
    const uint32_t G = 1u << g;
    if (g == 0 || nblk % (8u * G)) return b;
    const uint32_t x = b & 7u, j = b >> 3;
    return ((uint64_t)((j >> g) * 8u + x) << g) | (j & (G - 1u));
}

#if defined(__HIP_DEVICE_COMPILE__)
// The value of lane sel(i) in lane i (DPP lane exchange, CTRL its control
// word), 0 in the rows that ROW_MASK leaves out.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    int lo, hi;
    if constexpr (ROW_MASK == 0xF) {  // every lane written: no initial value needed
        lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    }
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
#endif

// Sum over the 64 lanes of a wave (float64, a fixed order), the same value in
// every lane.  Lane exchanges by DPP (vector ALU, no LDS round trips): quads
// (lane xor 1, xor 2), halves of a row (mirror), rows of 16 (mirror), then
// row 0 into row 1 and row 2 into row 3 (broadcast of lane 15), then rows 0-1
// into row 3 (broadcast of lane 31); the total is read from lane 63.
__device__ __forceinline__ double wave_sum(double v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
#else
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
#endif
}

#if defined(__HIP_DEVICE_COMPILE__)
// Lane exchange between two float64 registers: with H32, lanes 32-63 of x
// trade places with lanes 0-31 of y (v_permlane32_swap); otherwise the odd
// 16-lane rows of x with the even rows of y (v_permlane16_swap).
template <bool H32>
__device__ __forceinline__ void lane_swap(double &x, double &y)
{
    const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
    const uint32_t xl = (uint32_t)bx, xh = (uint32_t)(bx >> 32), yl = (uint32_t)by, yh = (uint32_t)(by >> 32);
    uint32_t lo0, lo1, hi0, hi1;
    if constexpr (H32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        lo0 = lo[0], lo1 = lo[1], hi0 = hi[0], hi1 = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        lo0 = lo[0], lo1 = lo[1], hi0 = hi[0], hi1 = hi[1];
    }
    x = __builtin_bit_cast(double, ((uint64_t)hi0 << 32) | lo0);
    y = __builtin_bit_cast(double, ((uint64_t)hi1 << 32) | lo1);
}
#endif

// Four wave sums at once (float64, a fixed order; the results are uniform).
// Two rounds of lane swaps leave, in each 16-lane row, one value's partials
// over the four rows (row 0: v0, row 1: v2, row 2: v1, row 3: v3); a
// reduction within rows finishes all four together: 6 swaps, 7 additions and
// 4 row steps instead of 4 x 6 exchange steps.
__device__ __forceinline__ void wave_sum4(double (&v)[4])
{
#if defined(__HIP_DEVICE_COMPILE__)
    lane_swap<true>(v[0], v[1]);
    double p = v[0] + v[1];  // lanes 0-31: v0's two halves, lanes 32-63: v1's
    lane_swap<true>(v[2], v[3]);
    double q = v[2] + v[3];  // the same for v2 and v3
    lane_swap<false>(p, q);
    double r = p + q;        // rows: v0, v2, v1, v3, each over the four rows
    r += dpp_f64<0xB1, 0xF>(r);   // quad_perm [1, 0, 3, 2]
    r += dpp_f64<0x4E, 0xF>(r);   // quad_perm [2, 3, 0, 1]
    r += dpp_f64<0x141, 0xF>(r);  // row_half_mirror
    r += dpp_f64<0x140, 0xF>(r);  // row_mirror: every lane of a row holds its total
    const uint64_t b = __builtin_bit_cast(uint64_t, r);
    const int lanes[4] = {0, 32, 16, 48};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lanes[j]);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lanes[j]);
        v[j] = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    }
#else
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = wave_sum(v[j]);
#endif
}

// Im <lambda|Z_j|psi> summed over the wave for the register slots j of mask
// (at least two of them): out[j], uniform; slots outside mask get 0.  Each
// amplitude's product is formed once and added, with the slot's sign, to
// every slot's float64 sum.
template <int R>
__device__ __forceinline__ void grad_z_members(const float2 (&a)[1 << R], const float2 (&l)[1 << R], uint32_t mask,
                                               double (&out)[R])
{
#pragma unroll
    for (int j = 0; j < R; ++j) out[j] = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        const double m = (double)__builtin_fmaf(l[i].x, a[i].y, -(l[i].y * a[i].x));  // Im(conj(l) a)
#pragma unroll
        for (int j = 0; j < R; ++j) out[j] += ((i >> j) & 1) ? -m : m;
    }
#pragma unroll
    for (int j0 = 0; j0 < R; j0 += 4) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (j0 + k < R && ((mask >> (j0 + k)) & 1u)) ? out[j0 + k] : 0.0;
        const uint32_t cm = (mask >> j0) & 15u;
        if (__builtin_popcount(cm) == 1) {  // one slot in this group of four
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) x = ((cm >> k) & 1u) ? v[k] : x;
            x = wave_sum(x);
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = ((cm >> k) & 1u) ? x : 0.0;
        } else if (cm) {
            wave_sum4(v);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (j0 + k < R) out[j0 + k] = v[k];
    }
}

// The gradient partials of op o (float64, summed over the wave): the one of
// its rotation, or, for a register diagonal folded from parameterised RZ
// rotations (OP_DREG with a gradient slot), one per member: the members are
// the register slots in o.a, member m (in slot order) has slot grad_slot + m.
// emit(slot, value) is called for each, with the same value in every lane.
template <int R, typename Emit>
__device__ __forceinline__ void grad_partials(const float2 (&a)[1 << R], const float2 (&l)[1 << R], const DevOp &o,
                                              uint32_t tid, uint64_t base, Emit &&emit)
{
    if (o.kind == OP_DREG) {
        uint32_t mask = (uint32_t)o.a;
        if (__builtin_popcount(mask) >= 2) {
            double v[R];
            grad_z_members<R>(a, l, mask, v);
#pragma unroll
            for (int j = 0, m = 0; j < R; ++j)
                if ((mask >> j) & 1u) emit(o.grad_slot + m++, v[j]);
            return;
        }
        for (int m = 0; mask; ++m, mask &= mask - 1) {
            double acc = 0.0;
            on_slot<R>(opaque(mask & (~mask + 1)), [&](auto J) __attribute__((always_inline)) {
                acc = grad_z_reg<R, std::decay_t<decltype(J)>::value>(a, l);
            });
            emit(o.grad_slot + m, wave_sum(acc));
        }
    } else {
        emit(o.grad_slot, wave_sum(grad_term<R>(a, l, o, tid, base)));
    }
}

// XOR swizzle of an 8-byte LDS slot: bits 5-9 and 10-14 of the tile position
// are folded into bits 0-4, so 32 lanes whose positions differ in bits with
// distinct residues mod 5 hit distinct bank pairs.  swz is linear over GF(2):
// for positions with disjoint bits swz(a | b) = swz(a) ^ swz(b), so a thread
// swizzles its thread-bit offset once and the register-bit offsets (uniform)
// are swizzled in scalar registers.
__device__ __forceinline__ uint32_t swz(uint32_t c) { return c ^ ((c >> 5) & 31u) ^ ((c >> 10) & 31u); }

// Swizzled LDS byte offsets of a stage layout: the thread's own part and the
// register-index parts (uniform).  An amplitude's slot is at byte toff ^ roff[i]
// (lds_ref): in bytes, so that each access costs one XOR and no shift.
template <int R>
__device__ __forceinline__ void stage_offsets(const DevStage *__restrict__ S, int w, uint32_t tid, uint32_t &toff,
                                              uint32_t (&roff)[1 << R])
{
    uint32_t t = 0;
    for (int b = 0; b < w; ++b) t |= ((tid >> b) & 1u) << S->thrpos[b];
    toff = swz(t) << 3;
    uint32_t r[1 << R];
    r[0] = 0;
#pragma unroll
    for (int i = 1; i < (1 << R); ++i) r[i] = r[i & (i - 1)] | (1u << S->regpos[__builtin_ctz(i)]);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) roff[i] = swz(r[i]) << 3;
}

// The LDS slot at a byte offset.
__device__ __forceinline__ float2 &lds_ref(float2 *lds, uint32_t byte)
{
    return *reinterpret_cast<float2 *>(reinterpret_cast<char *>(lds) + byte);
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
            for (int i = 0; i < NA; ++i) a[i] = lds_ref(lds, toff ^ roff[i]);
            for (int k = S->op_begin; k < S->op_end; ++k) apply_op<R, DAG>(a, ops[k], pool, tid, base);
            asm volatile("" : "+v"(toff));  // recompute the write-back addresses instead of keeping 2^R live
#pragma unroll
            for (int i = 0; i < NA; ++i) lds_ref(lds, toff ^ roff[i]) = a[i];
        }
        __syncthreads();
    }
}

}  // namespace qsv
