// Plan specialisation (paper Section 4.3, Step D: the computation of every
// partition is generated as code).  For each partition the lowered tables of
// the plan (its DevPart, register stages, ops and constant matrices) are
// written out as compile-time constants of a table type, followed by one
// kernel that instantiates spec_sweep (spec.cuh) for it.  rtc_driver.cpp
// compiles the programs and keeps the optional code-object cache.
#include <cstdio>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace qsv {

namespace {

// Floats of the matrix pool that an op of this kind reads.
int pool_floats(int kind, int R)
{
    switch (kind) {
    case OP_LAYER: return 2 * (1 << R) + 2 * R;
    case OP_DREG: return 2 * (1 << R);
    case OP_U2: return 32;
    default: return 8;
    }
}

void put_ints(std::string &s, const int32_t *v, int n)
{
    char b[16];
    s += '{';
    for (int i = 0; i < n; ++i) {
        std::snprintf(b, sizeof b, "%d,", v[i]);
        s += b;
    }
    s += '}';
}

void put_stage(std::string &s, const DevStage &st)
{
    char b[48];
    std::snprintf(b, sizeof b, "{%d,%d,", st.op_begin, st.op_end);
    s += b;
    put_ints(s, st.regpos, 8);
    s += ',';
    put_ints(s, st.thrpos, 16);
    s += "},\n";
}

void put_op(std::string &s, const DevOp &o)
{
    char b[160];
    std::snprintf(b, sizeof b, "{%d,%d,%d,%d,%d,%d,%d,%d},\n", o.kind, o.a, o.b, o.gen, o.mat, o.grad_slot, o.gate,
                  o.flags);
    s += b;
}

}  // namespace

bool specialise_reverse(const Plan &plan)
{
    return (plan.flags & QSV_PLAN_GRAD) && ((size_t)16 << plan.t) <= (size_t)64 * 1024;
}

namespace {

// The tables of partition p as namespace-scope constants and the table type
// qsv_gen::P<p> that refers to them (every float as an exact hexadecimal
// literal).  Matrices written from theta at apply time (dyn_mats) stay in the
// device pool; the others are copied in.
void put_tables(std::string &s, const Plan &plan, int p, const std::set<int32_t> &dyn_mats,
                const std::map<int32_t, const ParamDiag *> *expand = nullptr, const char *tag = "")
{
    char b[1024];
    const DevPart &P = plan.parts[p];
    DevPart lp = P;
    lp.stage_begin = 0;
    lp.stage_end = P.stage_end - P.stage_begin;
    std::vector<DevStage> stages;
    std::vector<DevOp> ops;
    std::vector<int> dyn;
    std::vector<float> pool;
    for (int si = P.stage_begin; si < P.stage_end; ++si) {
        DevStage st = plan.stages[si];
        const int k0 = st.op_begin, k1 = st.op_end;
        st.op_begin = (int32_t)ops.size();
        for (int k = k0; k < k1; ++k) {
            DevOp o = plan.ops[k];
            if (expand && o.kind == OP_DREG && o.grad_slot >= 0 && expand->count(o.mat)) {
                // a register diagonal folded from parameterised RZ rotations, as its
                // members' own rotations (in a forward kernel their separate
                // matrices take fewer loads than the 2^R entries)
                const ParamDiag &pd = *expand->at(o.mat);
                for (int m = 0; m < pd.n; ++m) {
                    DevOp e = o;
                    e.kind = OP_D1;
                    e.a = LOC_REG | pd.slot[m];
                    e.b = 0;
                    e.mat = pd.gmat[m];
                    e.grad_slot = o.grad_slot + m;
                    ops.push_back(e);
                    dyn.push_back(1);
                }
                continue;
            }
            const bool d = o.mat >= 0 && dyn_mats.count(o.mat) > 0;
            if (o.mat >= 0 && !d) {
                const int nf = pool_floats(o.kind, plan.R);
                const int off = (int)pool.size();
                for (int i = 0; i < nf; ++i)
                    pool.push_back((size_t)o.mat + i < plan.pool.size() ? plan.pool[o.mat + i] : 0.f);
                o.mat = off;
            }
            ops.push_back(o);
            dyn.push_back(d ? 1 : 0);
        }
        st.op_end = (int32_t)ops.size();
        stages.push_back(st);
    }
    // Namespace-scope constexpr arrays have internal linkage, so the compiler
    // folds every read of them into the code; static data members of the table
    // type would be inline (weak) symbols that it must load at run time.
    std::snprintf(b, sizeof b, "namespace qsv_gen {\nconstexpr qsv::DevPart part%s%d = {%d,%d,%d,%d,", tag, p,
                  lp.stage_begin, lp.stage_end, lp.t, lp.n_glb);
    s += b;
    put_ints(s, lp.tq, 16);
    s += ',';
    put_ints(s, lp.gq, 48);
    std::snprintf(b, sizeof b, "};\nconstexpr qsv::DevStage stages%s%d[] = {\n", tag, p);
    s += b;
    for (const DevStage &st : stages) put_stage(s, st);
    std::snprintf(b, sizeof b, "{}};\nconstexpr qsv::DevOp ops%s%d[] = {\n", tag, p);  // arrays end in an unused entry
    s += b;
    for (const DevOp &o : ops) put_op(s, o);
    std::snprintf(b, sizeof b, "{}};\nconstexpr bool dyn%s%d[] = {", tag, p);
    s += b;
    for (int d : dyn) s += d ? "1," : "0,";
    std::snprintf(b, sizeof b, "0};\nconstexpr float pool%s%d[] = {\n", tag, p);
    s += b;
    for (size_t i = 0; i < pool.size(); ++i) {
        std::snprintf(b, sizeof b, "%af,%s", (double)pool[i], (i % 8 == 7) ? "\n" : "");
        s += b;
    }
    std::snprintf(b, sizeof b,
                  "0.f};\nstruct P%s%d {\n    static constexpr int R = %d, LW = %d;\n"
                  "    static constexpr const qsv::DevPart &part = part%s%d;\n"
                  "    static constexpr const qsv::DevStage *stages = stages%s%d;\n"
                  "    static constexpr const qsv::DevOp *ops = ops%s%d;\n"
                  "    static constexpr const bool *dyn = dyn%s%d;\n"
                  "    static constexpr const float *pool = pool%s%d;\n};\n}  // namespace qsv_gen\n",
                  tag, p, plan.R, plan.LW, tag, p, tag, p, tag, p, tag, p, tag, p);
    s += b;
}

std::set<int32_t> dynamic_matrices(const Plan &plan)
{
    std::set<int32_t> dyn_mats;  // pool entries written from theta at apply time
    for (const ParamGate &g : plan.pgates) dyn_mats.insert(g.mat);
    for (const ParamDiag &d : plan.pdiags) dyn_mats.insert(d.mat);  // (member matrices are pgates' own)
    return dyn_mats;
}

}  // namespace

// Source of the program holding the specialised kernels qsv_spec_<p> (and,
// for gradient plans, qsv_rspec_<p>) of partitions [p0, p1).
std::string specialise_source(const Plan &plan, int p0, int p1, bool with_reverse)
{
    const std::set<int32_t> dyn_mats = dynamic_matrices(plan);
    // straight-line code: the gate bodies' plain arithmetic (see gates.cuh)
    std::string s = "#define QSV_PLAIN_ARITH 1\n#include \"spec.cuh\"\n";
    char b[1024];
    std::map<int32_t, const ParamDiag *> pdiag_of;  // folded RZ diagonals, by pool offset
    for (const ParamDiag &d : plan.pdiags) pdiag_of.emplace(d.mat, &d);
    for (int p = p0; p < p1; ++p) {
        // the forward kernel applies folded RZ diagonals as their members' own
        // rotations; the reverse walk keeps the folded form (fewer ops on psi
        // and lambda)
        put_tables(s, plan, p, dyn_mats, &pdiag_of);
        if (with_reverse) put_tables(s, plan, p, dyn_mats, nullptr, "r");
        std::snprintf(b, sizeof b,
                      "extern \"C\" __global__ __launch_bounds__(%d) void qsv_spec_%d(float2 *__restrict__ psi, "
                      "float2 *__restrict__ ckpt, const float *__restrict__ pool)\n"
                      "{\n    qsv::spec_sweep<qsv_gen::P%d>(psi, ckpt, pool);\n}\n",
                      1 << plan.LW, p, p);
        s += b;
        if (with_reverse) {
            std::snprintf(b, sizeof b,
                          "extern \"C\" __global__ __launch_bounds__(%d) void qsv_rspec_%d(const float2 *__restrict__ "
                          "psi, float2 *__restrict__ lam, const float *__restrict__ pool, double *__restrict__ gpart, "
                          "int64_t slot_stride)\n"
                          "{\n    qsv::spec_reverse<qsv_gen::Pr%d>(psi, lam, pool, gpart, slot_stride);\n}\n",
                          1 << plan.LW, p, p);
            s += b;
        }
    }
    return s;
}

// Source of the program holding qsv_bspec, the batched kernel of a batched
// plan specialised for its circuit structures (forward launches): the tables
// of every structure (the one partition of each circuit that does not share
// another's tables) and a walk that switches on the circuit's partition index
// to the structure's compiled-in stages.
std::string specialise_batched_source(const Plan &plan)
{
    const std::set<int32_t> dyn_mats = dynamic_matrices(plan);
    std::string s = "#define QSV_PLAIN_ARITH 1\n#include \"spec.cuh\"\n";
    std::vector<int> reps;
    for (const CircuitPlan &C : plan.circ)
        if (C.shares < 0) reps.push_back(C.part_begin);
    std::map<int32_t, const ParamDiag *> pdiag_of;  // folded RZ diagonals, by pool offset
    for (const ParamDiag &d : plan.pdiags) pdiag_of.emplace(d.mat, &d);
    for (int p : reps) put_tables(s, plan, p, dyn_mats, &pdiag_of);
    char b[512];
    s += "struct SpecWalk {\n"
         "    static __device__ __forceinline__ void forward(int pidx, const qsv::DevPart *, float2 *lds,\n"
         "        const qsv::DevStage *, const qsv::DevOp *, const float *__restrict__ cpool, uint32_t tid)\n"
         "    {\n        switch (pidx) {\n";
    for (int p : reps) {
        std::snprintf(b, sizeof b, "        case %d: qsv::spec_bforward<qsv_gen::P%d>(lds, cpool, tid); break;\n", p, p);
        s += b;
    }
    s += "        }\n    }\n"
         "    // never called: the specialised kernel runs forward launches only (the adjoint\n"
         "    // walk of a batched plan stays table-driven, from the forward's final states)\n"
         "    static __device__ __forceinline__ void adjoint(int, const qsv::DevPart *, float2 *,\n"
         "        const qsv::DevStage *, const qsv::DevOp *, const float *, int32_t, const qsv::DevGroup *,\n"
         "        const qsv::DevTerm *, const qsv::BatchArgs &, int, double *, uint32_t)\n"
         "    {\n";
    s += "    }\n};\n";
    std::snprintf(b, sizeof b,
                  "extern \"C\" __global__ __launch_bounds__(%d) void qsv_bspec(\n"
                  "    const qsv::DevPart *__restrict__ parts, const qsv::DevStage *__restrict__ stages,\n"
                  "    const qsv::DevOp *__restrict__ ops, const float *__restrict__ pool,\n", 1 << plan.LW);
    s += b;
    std::snprintf(b, sizeof b,
                  "    const int32_t *__restrict__ order, const int32_t *__restrict__ circ_part,\n"
                  "    const int64_t *__restrict__ circ_theta, const int64_t *__restrict__ circ_npar,\n"
                  "    const int32_t *__restrict__ param_off, const int32_t *__restrict__ param_slots,\n"
                  "    const int32_t *__restrict__ circ_pool_delta, const int32_t *__restrict__ circ_slot_delta,\n"
                  "    const qsv::DevGroup *__restrict__ groups, const qsv::DevTerm *__restrict__ terms,\n"
                  "    qsv::BatchArgs A)\n{\n");
    s += b;
    std::snprintf(b, sizeof b,
                  "    qsv::batched_body<%d, %d, SpecWalk>(parts, stages, ops, pool, order, circ_part, circ_theta,\n"
                  "        circ_npar, param_off, param_slots, circ_pool_delta, circ_slot_delta, groups, terms, A);\n}\n",
                  plan.R, plan.LW);
    s += b;
    return s;
}

}  // namespace qsv
