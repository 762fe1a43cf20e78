// The batched persistent kernel's body: many small circuits (n <= 14) with
// uneven depths, each run entirely on chip by one workgroup.  Shared by the
// library's table-driven kernel (batched.hip) and the kernels that
// qsv_plan_specialise generates for a batched plan, which differ only in how a
// circuit's register stages are walked (the Walk policy below).
//
// The grid holds one workgroup per compute unit.  A workgroup takes the next
// circuit from a device queue (circuits ordered by decreasing work, so the
// longest start first) until the queue is empty; every workgroup reaches that
// exit.  Per circuit:
//   forward  — |0..0> in LDS, the register stages of the circuit (one
//              partition covers the whole state), final state optionally
//              written out;
//   energy   — lambda = H psi in the last stage's register layout, reading the
//              partner amplitudes of each Pauli group from LDS; <H> reduced in
//              float64 in a fixed order;
//   adjoint  — stages walked backwards with psi and lambda both in registers,
//              remapped between stage layouts through LDS; for every
//              parameterised rotation Im <lambda|P|psi> is summed per wave
//              (float64) before U^dagger is applied to both states; the
//              circuit's gradient entries are then reduced in a fixed order.
#pragma once
#include "gates.cuh"

namespace qsv {

struct BatchArgs {
    int n_groups;
    int n_circuits;
    int n;
    float2 *psi_out;            // forward only: final states (may be null)
    const float2 *psi_in;       // adjoint only: final states of the forward (null: recompute them)
    double *energy;             // [n_circuits] (adjoint only)
    double *grad;               // [n_params]   (adjoint only)
    double *gpart;              // [n_slots][waves] scratch
    int *queue;
    int adjoint;
    uint64_t *wg_clock;         // null, or per workgroup the real-time clock at its start and at its exit
};

// Registers in the layout (toff, roff) -> LDS -> registers in the layout (toff2,
// roff2); offsets are already swizzled.
template <int R>
__device__ __forceinline__ void remap(float2 (&v)[1 << R], float2 *lds, bool active, uint32_t toff,
                                      const uint32_t (&roff)[1 << R], uint32_t toff2, const uint32_t (&roff2)[1 << R])
{
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) lds_ref(lds, toff ^ roff[i]) = v[i];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < (1 << R); ++i) v[i] = lds_ref(lds, toff2 ^ roff2[i]);
    }
}

// c with its sign bit flipped where bit 31 of sb is set.
__device__ __forceinline__ double flip_sign(double c, uint32_t sb)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, c) ^ ((uint64_t)sb << 32);
    return __builtin_bit_cast(double, b);
}

// f(integral_constant<int, i>) for i = B, B + S, ... below E, unrolled.
template <int B, int E, int S, typename F>
__device__ __forceinline__ void chunk_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        chunk_for<B + S, E, S>(static_cast<F &&>(f));
    }
}

// psi (a) and lambda = H psi (l) in the register layout (toff, roff), psi read
// from the LDS tile (positions are the qubits in order); the circuit's energy
// <psi|H|psi> (float64, waves in order) goes to *energy_out.
//
// Amplitude x_i of the thread has position tpos ^ rpos_i (thread part, and the
// uniform register part of slot i); swz is linear and its own inverse on
// these slots, so the partner x_i ^ X of a Pauli group sits at slot
// swz(tpos) ^ swz(rpos_i ^ X), and a term's sign (-1)^{|(x_i ^ X) & Z|} is the
// thread's parity of tpos & Z times the uniform parity of (rpos_i ^ X) & Z.
// The amplitudes are taken four at a time, each group and term record loaded
// once per four (not once per amplitude), with float64 sums per amplitude; a
// group of one term puts its sign on the partner amplitude, a longer group sums
// its terms per sign pattern over the four.  At 1024 threads this leaves a few
// per-circuit values spilled (outside the op loop); the gradient from final
// states still ran 4 % faster.
template <int R, int LW>
__device__ __forceinline__ void batch_energy(const float2 *lds, bool active, uint32_t toff,
                                             const uint32_t (&roff)[1 << R], const DevGroup *__restrict__ groups,
                                             const DevTerm *__restrict__ terms, int n_groups, float2 (&a)[1 << R],
                                             float2 (&l)[1 << R], double *s_red, double *energy_out, uint32_t tid)
{
    constexpr int NA = 1 << R, WAVES = (1 << LW) / 64, C = NA < 4 ? NA : 4;
    const uint32_t tslot = toff >> 3, tpos = swz(tslot);
    uint32_t rpos[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        rpos[i] = swz(roff[i] >> 3);
        a[i] = active ? lds[tslot ^ (roff[i] >> 3)] : float2{0.f, 0.f};
        l[i] = float2{0.f, 0.f};
    }
    double e_part = 0.0;
    if (active) {
        chunk_for<0, NA, C>([&](auto c0c) __attribute__((always_inline)) {
            constexpr int c0 = decltype(c0c)::value;
            double lr[C], li[C];
#pragma unroll
            for (int j = 0; j < C; ++j) lr[j] = li[j] = 0.0;
            for (int g = 0; g < n_groups; ++g) {
                const DevGroup G = groups[g];
                const uint32_t xm = (uint32_t)G.x_mask;
                if (G.term_end - G.term_begin == 1) {
                    // one term (most groups): its sign goes onto the partner amplitude
                    const DevTerm T = terms[G.term_begin];
                    const uint32_t z = (uint32_t)T.z_mask;
                    const uint32_t tsb = (uint32_t)__popc(tpos & z) << 31;
#pragma unroll
                    for (int j = 0; j < C; ++j) {
                        const uint32_t sb =
                            tsb ^ (uint32_t)__builtin_amdgcn_readfirstlane((int)((uint32_t)__popc((rpos[c0 + j] ^ xm) & z) << 31));
                        const float2 py = lds[tslot ^ swz(rpos[c0 + j] ^ xm)];
                        const double qx = (double)__uint_as_float(__float_as_uint(py.x) ^ sb);
                        const double qy = (double)__uint_as_float(__float_as_uint(py.y) ^ sb);
                        lr[j] += T.cre * qx - T.cim * qy;
                        li[j] += T.cre * qy + T.cim * qx;
                    }
                    continue;
                }
                double wr[C], wi[C];
#pragma unroll
                for (int j = 0; j < C; ++j) wr[j] = wi[j] = 0.0;
                if constexpr (C == 4) {
                    // The chunk's amplitudes differ in register bits 0 and 1 (position
                    // masks r1, r2), so a term's signs over the chunk are its sign at
                    // amplitude c0 times chi_p(j) = (-1)^{|j & p|}, p = the term's Z
                    // bits at r1 and r2 (uniform).  The terms are summed per pattern p
                    // (b[p]), then w_j = sum_p chi_p(j) b[p].
                    const uint32_t r1 = rpos[c0 + 1] ^ rpos[c0], r2 = rpos[c0 + 2] ^ rpos[c0];
                    double br[4] = {0.0, 0.0, 0.0, 0.0}, bi[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int k = G.term_begin; k < G.term_end; ++k) {
                        const DevTerm T = terms[k];
                        const uint32_t z = (uint32_t)T.z_mask;
                        // the sign at amplitude c0 as a float64 sign bit: the thread's
                        // part, then the uniform part
                        const uint32_t sb =
                            ((uint32_t)__popc(tpos & z) << 31) ^
                            (uint32_t)__builtin_amdgcn_readfirstlane((int)((uint32_t)__popc((rpos[c0] ^ xm) & z) << 31));
                        const int pat = __builtin_amdgcn_readfirstlane((int)(((z & r1) ? 1u : 0u) | ((z & r2) ? 2u : 0u)));
                        const double ar = flip_sign(T.cre, sb);
                        if (pat == 0) br[0] += ar;
                        else if (pat == 1) br[1] += ar;
                        else if (pat == 2) br[2] += ar;
                        else br[3] += ar;
                        if (T.cim != 0.0) {
                            const double ai = flip_sign(T.cim, sb);
                            if (pat == 0) bi[0] += ai;
                            else if (pat == 1) bi[1] += ai;
                            else if (pat == 2) bi[2] += ai;
                            else bi[3] += ai;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool neg = __builtin_popcount(j & q) & 1;
                            wr[j] += neg ? -br[q] : br[q];
                            wi[j] += neg ? -bi[q] : bi[q];
                        }
                    }
                } else {
                    for (int k = G.term_begin; k < G.term_end; ++k) {
                        const DevTerm T = terms[k];
                        const uint32_t z = (uint32_t)T.z_mask;
                        // the sign as a float64 sign bit: the thread's part, then the
                        // uniform part of each amplitude (scalar registers)
                        const uint32_t tsb = (uint32_t)__popc(tpos & z) << 31;
#pragma unroll
                        for (int j = 0; j < C; ++j) {
                            const uint32_t sb = tsb ^ (uint32_t)__builtin_amdgcn_readfirstlane(
                                                          (int)((uint32_t)__popc((rpos[c0 + j] ^ xm) & z) << 31));
                            wr[j] += flip_sign(T.cre, sb);
                            if (T.cim != 0.0) wi[j] += flip_sign(T.cim, sb);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    // (also for X = 0: a select between this read and a[] would put a[] in memory)
                    const float2 py = lds[tslot ^ swz(rpos[c0 + j] ^ xm)];
                    lr[j] += wr[j] * py.x - wi[j] * py.y;
                    li[j] += wr[j] * py.y + wi[j] * py.x;
                }
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                l[c0 + j] = float2{(float)lr[j], (float)li[j]};
                e_part += (double)a[c0 + j].x * lr[j] + (double)a[c0 + j].y * li[j];
            }
        });
    }
    e_part = wave_sum(e_part);
    if ((tid & 63) == 0) s_red[tid >> 6] = e_part;
    __syncthreads();
    if (tid == 0) {
        double e = 0.0;
        for (int v = 0; v < WAVES; ++v) e += s_red[v];
        *energy_out = e;
    }
}

// The table-driven walk: the circuit's stage and op tables read at run time.
template <int R, int LW>
struct TableWalk {
    static __device__ __forceinline__ void forward(int, const DevPart *__restrict__ P, float2 *lds,
                                                   const DevStage *__restrict__ stages,
                                                   const DevOp *__restrict__ ops, const float *__restrict__ cpool,
                                                   uint32_t tid)
    {
        run_stages<R, false>(lds, stages, ops, cpool, P->stage_begin, P->stage_end, P->t - R, tid, 0);
    }

    static __device__ __forceinline__ void adjoint(int, const DevPart *__restrict__ P, float2 *lds,
                                                   const DevStage *__restrict__ stages,
                                                   const DevOp *__restrict__ ops, const float *__restrict__ cpool,
                                                   int32_t slot_delta, const DevGroup *__restrict__ groups,
                                                   const DevTerm *__restrict__ terms, const BatchArgs &A, int c,
                                                   double *s_red, uint32_t tid)
    {
        constexpr int NA = 1 << R, WAVES = (1 << LW) / 64;
        const int w = P->t - R;
        const bool active = tid < (1u << w);
        const int wave = tid >> 6;
        // lambda = H psi and the energy, in the last stage's layout
        const int s_last = P->stage_end - 1;
        uint32_t toff, roff[NA];
        stage_offsets<R>(stages + s_last, w, tid, toff, roff);
        float2 a[NA], l[NA];
        batch_energy<R, LW>(lds, active, toff, roff, groups, terms, A.n_groups, a, l, s_red, A.energy + c, tid);
        // reverse walk over the stages
        for (int s = s_last; s >= P->stage_begin; --s) {
            if (s != s_last) {  // remap psi, then lambda, from the layout of stage s+1 to that of stage s
                uint32_t toff2, roff2[NA];
                stage_offsets<R>(stages + s, w, tid, toff2, roff2);
                remap<R>(a, lds, active, toff, roff, toff2, roff2);
                remap<R>(l, lds, active, toff, roff, toff2, roff2);
                toff = toff2;
#pragma unroll
                for (int i = 0; i < NA; ++i) roff[i] = roff2[i];
            }
            const DevStage *__restrict__ S = stages + s;
            for (int k = S->op_end - 1; k >= S->op_begin; --k) {
                const DevOp o = ops[k];
                if (o.grad_slot >= 0)
                    grad_partials<R>(a, l, o, tid, 0, [&](int32_t slot, double v) __attribute__((always_inline)) {
                        if ((tid & 63) == 0) A.gpart[(int64_t)(slot + slot_delta) * WAVES + wave] = v;
                    });
                // one dispatch, then psi and lambda one after the other (a
                // dispatch per array cost 9 % more time)
                apply_ops<R, true, true>(o, cpool, tid, 0, a, l);
            }
        }
    }
};

// Walk is a policy with two static device functions for circuit c, whose one
// partition is parts[pidx] and whose matrices sit at cpool (the shared tables'
// offsets plus the circuit's pool delta):
//   forward(pidx, P, lds, stages, ops, cpool, tid): the register stages on the
//       LDS tile, ending with a barrier;
//   adjoint(pidx, P, lds, stages, ops, cpool, slot_delta, groups, terms, A, c,
//       s_red, tid): energy and lambda from the LDS tile (batch_energy), then
//       the reverse walk writing gradient partials to A.gpart.
template <int R, int LW, class Walk>
__device__ __forceinline__ void batched_body(
    const DevPart *__restrict__ parts, const DevStage *__restrict__ stages, const DevOp *__restrict__ ops,
    const float *__restrict__ pool, const int32_t *__restrict__ order, const int32_t *__restrict__ circ_part,
    const int64_t *__restrict__ circ_theta, const int64_t *__restrict__ circ_npar,
    const int32_t *__restrict__ param_off, const int32_t *__restrict__ param_slots,
    const int32_t *__restrict__ circ_pool_delta, const int32_t *__restrict__ circ_slot_delta,
    const DevGroup *__restrict__ groups, const DevTerm *__restrict__ terms, const BatchArgs &A)
{
    constexpr int WAVES = (1 << LW) / 64;
    extern __shared__ float2 lds[];
    __shared__ int s_item;
    __shared__ double s_red[WAVES];
    const uint32_t tid = threadIdx.x;
    if (A.wg_clock && tid == 0) A.wg_clock[2 * blockIdx.x] = __builtin_amdgcn_s_memrealtime();
    while (true) {
        if (tid == 0) s_item = atomicAdd(A.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // the same for every thread
        __syncthreads();
        if (item >= A.n_circuits) break;
        const int c = order[item];
        // circuits of the same structure share their tables: this circuit's own
        // matrices and gradient slots sit at a constant offset from the ones the
        // tables name
        const int pidx = circ_part[c];
        const DevPart *__restrict__ P = parts + pidx;
        const float *__restrict__ cpool = pool + circ_pool_delta[c];
        const int32_t slot_delta = circ_slot_delta[c];
        const uint32_t dim = 1u << P->t;
        if (A.psi_in) {  // the forward's final state (positions are the qubits in order)
            const float2 *src = A.psi_in + (uint64_t)c * dim;
            for (uint32_t x = tid; x < dim; x += (1u << LW)) lds[swz(x)] = src[x];
            __syncthreads();
        } else {  // forward from |0..0>
            for (uint32_t x = tid; x < dim; x += (1u << LW)) lds[swz(x)] = float2{x == 0 ? 1.f : 0.f, 0.f};
            __syncthreads();
            Walk::forward(pidx, P, lds, stages, ops, cpool, tid);
        }
        if (A.psi_out) {  // the tile is the whole state and its positions are the qubits in order
            float2 *dst = A.psi_out + (uint64_t)c * dim;
            for (uint32_t x = tid; x < dim; x += (1u << LW)) dst[x] = lds[swz(x)];
        }
        if (!A.adjoint) {
            __syncthreads();
            continue;
        }
        Walk::adjoint(pidx, P, lds, stages, ops, cpool, slot_delta, groups, terms, A, c, s_red, tid);
        // this circuit's gradient entries: slots in slot order, waves in order
        __threadfence_block();
        __syncthreads();
        const int64_t p0 = circ_theta[c], np = circ_npar[c];
        for (int64_t p = tid; p < np; p += (1 << LW)) {
            double acc = 0.0;
            for (int32_t k = param_off[p0 + p]; k < param_off[p0 + p + 1]; ++k)
                for (int v = 0; v < WAVES; ++v) acc += A.gpart[(int64_t)param_slots[k] * WAVES + v];
            A.grad[p0 + p] = acc;
        }
        __syncthreads();
    }
    if (A.wg_clock && tid == 0) A.wg_clock[2 * blockIdx.x + 1] = __builtin_amdgcn_s_memrealtime();
}

}  // namespace qsv
