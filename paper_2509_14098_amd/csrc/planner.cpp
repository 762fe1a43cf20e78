// Host planner: gate classification, contraction graph, closeness centrality,
// greedy frontier partitioning (two levels) and lowering to device tables.
//
// Paper references (arXiv:2509.14098):
//   Section 4.1, Fig. 4  contraction graph and critical-path lengths l_v
//   Section 4.2, Eq. 10-13, Fig. 5  closeness centrality and the forward
//                        frontier sweep with its two locality exemptions
//   Section 4.3, Fig. 6  partition tree, tiles and on-chip buffers
// All graph quantities are integers; centralities are compared exactly.
#include <algorithm>
#include <cmath>
#include <complex>
#include <array>
#include <cstring>
#include <functional>
#include <set>
#include <stdexcept>
#include <unordered_map>

#include "internal.h"

namespace qsv {

using cd = std::complex<double>;

static int popc(uint64_t x) { return __builtin_popcountll(x); }

static int arity(int kind)
{
    if ((kind >= QSV_H && kind <= QSV_U3) || kind == QSV_MAT1) return 1;
    if ((kind >= QSV_CX && kind <= QSV_RZZ) || kind == QSV_MAT2) return 2;
    return 0;
}

static bool is_rotation(int kind) { return kind == QSV_RX || kind == QSV_RY || kind == QSV_RZ || kind == QSV_RZZ; }

std::string validate_gate(const qsv_gate &g, int n, int64_t)
{
    int k = arity(g.kind);
    if (k == 0) return "unknown gate kind " + std::to_string(g.kind);
    if (g.q0 < 0 || g.q0 >= n) return "qubit q0 out of range";
    if (k == 2 && (g.q1 < 0 || g.q1 >= n)) return "qubit q1 out of range";
    if (k == 2 && g.q1 == g.q0) return "two-qubit gate on one qubit";
    if (g.param >= 0 && !is_rotation(g.kind)) return "param on a non-rotation gate";
    return "";
}

// Gate matrix in float64 (textbook / OpenQASM 2 definitions), row-major, local
// index j = b(q0) + 2 b(q1) for two-qubit gates.
static void fixed_matrix(const qsv_gate &g, cd m[16])
{
    for (int i = 0; i < 16; ++i) m[i] = 0.0;
    const double a = g.angle[0];
    const double h = 1.0 / std::sqrt(2.0);
    const cd I(0.0, 1.0);
    switch (g.kind) {
    case QSV_H: m[0] = h; m[1] = h; m[2] = h; m[3] = -h; break;
    case QSV_X: m[1] = 1.0; m[2] = 1.0; break;
    case QSV_Y: m[1] = -I; m[2] = I; break;
    case QSV_Z: m[0] = 1.0; m[3] = -1.0; break;
    case QSV_S: m[0] = 1.0; m[3] = I; break;
    case QSV_SDG: m[0] = 1.0; m[3] = -I; break;
    case QSV_T: m[0] = 1.0; m[3] = std::exp(I * (M_PI / 4.0)); break;
    case QSV_TDG: m[0] = 1.0; m[3] = std::exp(-I * (M_PI / 4.0)); break;
    case QSV_SX: m[0] = cd(0.5, 0.5); m[1] = cd(0.5, -0.5); m[2] = cd(0.5, -0.5); m[3] = cd(0.5, 0.5); break;
    case QSV_RX: m[0] = std::cos(a / 2); m[1] = -I * std::sin(a / 2); m[2] = -I * std::sin(a / 2); m[3] = std::cos(a / 2); break;
    case QSV_RY: m[0] = std::cos(a / 2); m[1] = -std::sin(a / 2); m[2] = std::sin(a / 2); m[3] = std::cos(a / 2); break;
    case QSV_RZ: m[0] = std::exp(-I * (a / 2)); m[3] = std::exp(I * (a / 2)); break;
    case QSV_P: m[0] = 1.0; m[3] = std::exp(I * a); break;
    case QSV_U3: {
        double t = g.angle[0], p = g.angle[1], l = g.angle[2];
        m[0] = std::cos(t / 2);
        m[1] = -std::exp(I * l) * std::sin(t / 2);
        m[2] = std::exp(I * p) * std::sin(t / 2);
        m[3] = std::exp(I * (p + l)) * std::cos(t / 2);
        break;
    }
    case QSV_MAT1: for (int i = 0; i < 4; ++i) m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]); break;
    case QSV_CX: m[0] = 1.0; m[10] = 1.0; m[1 * 4 + 3] = 1.0; m[3 * 4 + 1] = 1.0; break;
    case QSV_CY: m[0] = 1.0; m[10] = 1.0; m[1 * 4 + 3] = -I; m[3 * 4 + 1] = I; break;
    case QSV_CZ: m[0] = 1.0; m[5] = 1.0; m[10] = 1.0; m[15] = -1.0; break;
    case QSV_CP: m[0] = 1.0; m[5] = 1.0; m[10] = 1.0; m[15] = std::exp(I * a); break;
    case QSV_SWAP: m[0] = 1.0; m[1 * 4 + 2] = 1.0; m[2 * 4 + 1] = 1.0; m[15] = 1.0; break;
    case QSV_RZZ:
        m[0] = std::exp(-I * (a / 2)); m[5] = std::exp(I * (a / 2)); m[10] = std::exp(I * (a / 2)); m[15] = std::exp(-I * (a / 2));
        break;
    case QSV_MAT2: for (int i = 0; i < 16; ++i) m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]); break;
    default: break;
    }
}

GateMeta classify(const qsv_gate &g)
{
    GateMeta r;
    r.nq = arity(g.kind);
    r.q[0] = g.q0;
    r.q[1] = r.nq == 2 ? g.q1 : -1;
    r.qmask = (1ull << g.q0) | (r.nq == 2 ? (1ull << g.q1) : 0ull);
    r.param = g.param >= 0;
    if (r.param) {  // structure for a generic angle; matrix formed on the device
        switch (g.kind) {
        case QSV_RX: r.op = OP_U1; r.req = r.qmask; r.gen = GEN_X; r.flops = 14; break;
        case QSV_RY: r.op = OP_R1; r.req = r.qmask; r.gen = GEN_Y; r.flops = 6; break;
        case QSV_RZ: r.op = OP_D1; r.req = 0; r.gen = GEN_Z; r.flops = 6; break;
        default: r.op = OP_D2; r.req = 0; r.gen = GEN_ZZ; r.flops = 6; break;  // RZZ
        }
        return r;
    }
    cd m[16];
    fixed_matrix(g, m);
    for (int i = 0; i < 16; ++i) { r.m[2 * i] = m[i].real(); r.m[2 * i + 1] = m[i].imag(); }
    if (r.nq == 1) {
        bool diag = m[1] == 0.0 && m[2] == 0.0;
        bool real = m[0].imag() == 0 && m[1].imag() == 0 && m[2].imag() == 0 && m[3].imag() == 0;
        if (diag) { r.op = OP_D1; r.req = 0; r.flops = 6; }
        else if (real) { r.op = OP_R1; r.req = r.qmask; r.flops = 6; }
        else { r.op = OP_U1; r.req = r.qmask; r.flops = 14; }
        return r;
    }
    auto at = [&](int i, int j) { return m[i * 4 + j]; };
    bool diag = true;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if (i != j && at(i, j) != 0.0) diag = false;
    if (diag) {
        bool cz = at(0, 0) == 1.0 && at(1, 1) == 1.0 && at(2, 2) == 1.0 && at(3, 3) == -1.0;
        r.op = cz ? OP_CZ : OP_D2;
        r.req = 0;
        r.flops = cz ? 0 : 6;
        return r;
    }
    // controlled structure: identity while the control is 0 and no mixing of
    // the control value (Section 4.2 second exemption)
    for (int c = 0; c < 2; ++c) {
        int z[2], o[2];
        if (c == 0) { z[0] = 0; z[1] = 2; o[0] = 1; o[1] = 3; }
        else { z[0] = 0; z[1] = 1; o[0] = 2; o[1] = 3; }
        bool mixing = false, ident = true;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                if (at(z[a], o[b]) != 0.0 || at(o[a], z[b]) != 0.0) mixing = true;
                if (at(z[a], z[b]) != (a == b ? 1.0 : 0.0)) ident = false;
            }
        if (!mixing && ident) {
            r.ctrl = r.q[c];
            r.tgt = r.q[1 - c];
            r.req = 1ull << r.tgt;
            cd u[4] = {at(o[0], o[0]), at(o[0], o[1]), at(o[1], o[0]), at(o[1], o[1])};
            for (int i = 0; i < 4; ++i) { r.m[2 * i] = u[i].real(); r.m[2 * i + 1] = u[i].imag(); }
            for (int i = 8; i < 32; ++i) r.m[i] = 0;
            bool x = u[0] == 0.0 && u[3] == 0.0 && u[1] == 1.0 && u[2] == 1.0;
            r.op = x ? OP_CX : OP_CU;
            r.flops = x ? 0 : 7;
            return r;
        }
    }
    bool swap = true;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            int pj = (j == 1) ? 2 : (j == 2) ? 1 : j;
            if (at(i, j) != (i == pj ? 1.0 : 0.0)) swap = false;
        }
    r.op = swap ? OP_SWAP : OP_U2;
    r.req = r.qmask;
    r.flops = swap ? 0 : 30;
    return r;
}

// ---------------------------------------------------------------------------
// Greedy frontier partition of the gates `sub` (in circuit order) into parts
// of at most k required-local qubits.
//
// Contraction graph: node 0 is the incoming state tensor, node i+1 the gate
// sub[i]; every qubit of a gate adds an edge from the previous tensor on that
// qubit.  l(0) = 0, l(v) = 1 + max l(pred).  RN(v) = all downstream nodes,
// dist(v) = sum_{w in RN(v)} (l_w - l_v) (the telescoped form of Eq. 12-13),
// CC(v) = |RN|^2 / (N dist) (Eq. 10 with the Wasserman-Faust factor) or 0 when
// RN is empty.  Frontier sweep: among the gates whose predecessors are all
// placed, take the one of highest CC (then lower l, then lower index) whose
// required qubits fit; grow S by all its qubits (those in `allowed`) if they
// fit, else by the required ones; close the part when nothing fits.  The
// returned S are not padded.
// ---------------------------------------------------------------------------
std::vector<Part> greedy_partition(int n, const std::vector<GateMeta> &meta, const std::vector<int> &sub, int k,
                                   uint64_t allowed)
{
    const int G = (int)sub.size();
    std::vector<Part> parts;
    if (G == 0) return parts;
    const int N = G + 1;
    std::vector<int> pred0(N, -1), pred1(N, -1);
    std::vector<std::vector<int>> succ(N);
    std::vector<int> last(n, 0), l(N, 0);
    for (int i = 0; i < G; ++i) {
        const GateMeta &g = meta[sub[i]];
        int v = i + 1, u0 = last[g.q[0]], u1 = g.nq == 2 ? last[g.q[1]] : -1;
        pred0[v] = u0;
        succ[u0].push_back(v);
        if (u1 >= 0 && u1 != u0) { pred1[v] = u1; succ[u1].push_back(v); }
        l[v] = 1 + std::max(l[u0], u1 >= 0 ? l[u1] : 0);
        last[g.q[0]] = v;
        if (g.nq == 2) last[g.q[1]] = v;
    }
    // reachable sets as bitsets, filled from the last node backwards.  The sum
    // of l over a set is taken bit plane by bit plane: sum_w l_w =
    // sum_b 2^b |RN(v) & {w : bit b of l_w set}|, so no set bit is visited.
    const int words = (N + 63) / 64;
    std::vector<uint64_t> rn((size_t)N * words, 0);
    std::vector<int64_t> size(N, 0), dist(N, 0);
    int planes = 1;
    for (int v = 0; v < N; ++v)
        while ((l[v] >> planes) != 0) ++planes;
    std::vector<uint64_t> plane((size_t)planes * words, 0);
    for (int v = 0; v < N; ++v)
        for (int b = 0; b < planes; ++b)
            if ((l[v] >> b) & 1) plane[(size_t)b * words + (v >> 6)] |= 1ull << (v & 63);
    for (int v = N - 1; v >= 0; --v) {
        uint64_t *rv = &rn[(size_t)v * words];
        for (int c : succ[v]) {
            const uint64_t *rc = &rn[(size_t)c * words];
            for (int w = 0; w < words; ++w) rv[w] |= rc[w];
            rv[c >> 6] |= 1ull << (c & 63);
        }
    }
    for (int v = 0; v < N; ++v) {
        const uint64_t *rv = &rn[(size_t)v * words];
        int64_t cnt = 0, suml = 0;
        for (int w = 0; w < words; ++w) cnt += popc(rv[w]);
        for (int b = 0; b < planes; ++b) {
            const uint64_t *pb = &plane[(size_t)b * words];
            int64_t c = 0;
            for (int w = 0; w < words; ++w) c += popc(rv[w] & pb[w]);
            suml += c << b;
        }
        size[v] = cnt;
        dist[v] = suml - cnt * (int64_t)l[v];
    }
    // exact comparison of (CC desc, l asc, index asc)
    auto better = [&](int a, int b) {
        if (size[a] == 0 || size[b] == 0) {
            if (size[a] != 0) return true;
            if (size[b] != 0) return false;
        } else {
            unsigned __int128 lhs = (unsigned __int128)(size[a] * size[a]) * (uint64_t)dist[b];
            unsigned __int128 rhs = (unsigned __int128)(size[b] * size[b]) * (uint64_t)dist[a];
            if (lhs != rhs) return lhs > rhs;
        }
        if (l[a] != l[b]) return l[a] < l[b];
        return a < b;
    };
    std::vector<int> missing(N, 0), ready;
    for (int v = 1; v < N; ++v) {
        missing[v] = (pred0[v] > 0) + (pred1[v] > 0);
        if (missing[v] == 0) ready.push_back(v);
    }
    int placed = 0;
    while (placed < G) {
        Part part;
        while (true) {
            int best = -1;
            for (int v : ready) {
                const GateMeta &g = meta[sub[v - 1]];
                if (popc(part.S | g.req) <= k && (best < 0 || better(v, best))) best = v;
            }
            if (best < 0) break;
            const GateMeta &g = meta[sub[best - 1]];
            uint64_t grow = g.qmask & allowed;
            part.S = popc(part.S | grow) <= k ? (part.S | grow) : (part.S | g.req);
            part.gates.push_back(sub[best - 1]);
            ready.erase(std::find(ready.begin(), ready.end(), best));
            for (int w : succ[best])
                if (--missing[w] == 0) ready.push_back(w);
            ++placed;
        }
        if (part.gates.empty()) throw std::logic_error("partitioner made no progress");
        parts.push_back(std::move(part));
    }
    return parts;
}

// ---------------------------------------------------------------------------
// Lowering
// ---------------------------------------------------------------------------
static uint64_t pad_low(uint64_t S, int n, int k)
{
    for (int q = 0; q < n && popc(S) < k; ++q) S |= 1ull << q;
    return S;
}

// Register/lane/wave layout of a stage.  Register slots take the stage's
// required qubits, padded with the highest free tile positions; lanes 0..4
// take free positions with distinct residues mod 5 where possible, so that the
// XOR-swizzled LDS addresses of a half-wave fall into distinct 8-byte bank
// slots; the other thread bits take the remaining positions in order.
static void stage_layout(uint32_t reg_posmask, int t, int R, int w, DevStage &st)
{
    std::vector<int> reg, freep;
    for (int p = 0; p < t; ++p) ((reg_posmask >> p) & 1 ? reg : freep).push_back(p);
    while ((int)reg.size() < R) {
        reg.push_back(freep.back());
        freep.pop_back();
    }
    std::sort(reg.begin(), reg.end());
    for (int j = 0; j < R; ++j) st.regpos[j] = reg[j];
    std::vector<int> lanes;
    std::vector<bool> used(freep.size(), false);
    int want = std::min(5, w);
    bool res[5] = {false, false, false, false, false};
    for (size_t i = 0; i < freep.size() && (int)lanes.size() < want; ++i)
        if (!res[freep[i] % 5]) { res[freep[i] % 5] = true; lanes.push_back(freep[i]); used[i] = true; }
    for (size_t i = 0; i < freep.size() && (int)lanes.size() < want; ++i)
        if (!used[i]) { lanes.push_back(freep[i]); used[i] = true; }
    for (size_t i = 0; i < freep.size(); ++i)
        if (!used[i]) lanes.push_back(freep[i]);
    for (int b = 0; b < w; ++b) st.thrpos[b] = lanes[b];
}

// ---------------------------------------------------------------------------
// Register-stage lowering with diagonal folding.
//
// Every 2x2 unitary factors exactly as U = D1 R D2 with D1, D2 diagonal and R
// real ([[c, -s], [s, c]]); U3(t, p, l) = P(p) RY(t) P(l) is the familiar case.
// Inside a stage, diagonal factors and diagonal gates on register qubits
// commute with rotations on other qubits, so they are accumulated into one
// diagonal over the register index (2^R complex entries, the same for every
// thread) and applied as one complex multiply per amplitude.  The pending
// block is kept as  Dpost * (rotations on distinct qubits) * Dpre  (Dpre
// first).  A CX or SWAP between register qubits is crossed by permuting the
// diagonal's entries.  Parameterised gates (matrices formed on the device) and
// ops on thread or tile-index qubits that do not commute with the block end it.
// ---------------------------------------------------------------------------
namespace {

struct Diag {
    std::vector<cd> d;
    explicit Diag(int na = 0) : d(na, cd(1.0, 0.0)) {}
    bool identity() const
    {
        for (auto &v : d)
            if (v != cd(1.0, 0.0)) return false;
        return true;
    }
    bool depends_on(int j) const
    {
        for (size_t i = 0; i < d.size(); ++i)
            if (d[i] != d[i ^ (size_t(1) << j)]) return true;
        return false;
    }
};

// U = D1 R D2, with D2 = diag(1, e^{i b2}); false when U is not (numerically) unitary-shaped.
bool split_unitary(const double *m, cd &d1a, cd &d1b, double &c, double &sn, cd &d2b)
{
    const cd a(m[0], m[1]), b(m[2], m[3]), cc(m[4], m[5]), d(m[6], m[7]);
    c = std::abs(a);
    sn = std::abs(cc);
    if (std::abs(c * c + sn * sn - 1.0) > 1e-12) return false;
    double al1, al2, be2;
    if (c > 1e-300 && sn > 1e-300) {
        al1 = std::arg(a);
        al2 = std::arg(cc);
        be2 = std::arg(-b) - al1;
    } else if (sn <= 1e-300) {  // diagonal: handled as a diagonal gate, not here
        return false;
    } else {                    // anti-diagonal: R = [[0, -1], [1, 0]]
        al1 = 0.0;
        al2 = std::arg(cc);
        be2 = std::arg(-b);
    }
    d1a = std::polar(1.0, al1);
    d1b = std::polar(1.0, al2);
    d2b = std::polar(1.0, be2);
    // reconstruct and check
    const cd ra = d1a * c, rb = -d1a * sn * d2b, rc = d1b * sn, rd = d1b * c * d2b;
    const double err = std::abs(ra - a) + std::abs(rb - b) + std::abs(rc - cc) + std::abs(rd - d);
    return err < 1e-12;
}

struct StageLowering {
    Plan &P;
    const GateMeta *meta;
    const std::vector<int32_t> &mat_of;
    int R, NA;
    std::function<int32_t(int)> loc;
    const CircuitPlan &C;
    Diag pre, post;
    std::vector<std::pair<int, std::array<double, 4>>> rots;  // (register slot, real matrix)
    uint32_t rot_mask = 0;
    // parameterised RZ rotations on register slots, pending as one register
    // diagonal formed on the device (they commute with each other and with
    // everything that acts on other slots or only diagonally)
    std::vector<std::pair<int, int>> prz;  // (register slot, gate)
    uint32_t prz_mask = 0;

    StageLowering(Plan &P_, const std::vector<int32_t> &mo, int R_, std::function<int32_t(int)> loc_,
                  const CircuitPlan &C_)
        : P(P_), meta(P_.meta.data()), mat_of(mo), R(R_), NA(1 << R_), loc(std::move(loc_)), C(C_), pre(1 << R_),
          post(1 << R_)
    {
    }

    static bool is_reg(int32_t l) { return (l & LOC_MASK) == LOC_REG; }

    DevOp base_op(int kind, int gate)
    {
        DevOp o;
        std::memset(&o, 0, sizeof(o));
        o.kind = kind;
        o.gate = gate;
        o.grad_slot = -1;
        o.mat = -1;
        return o;
    }
    void add(const DevOp &o, double flops)
    {
        P.ops.push_back(o);
        P.flops += flops * std::ldexp(1.0, P.n);
    }
    void emit_diag(Diag &D, int gate)
    {
        if (D.identity()) return;
        DevOp o = base_op(OP_DREG, gate);
        o.mat = (int32_t)P.pool.size();
        for (auto &v : D.d) {
            P.pool.push_back((float)v.real());
            P.pool.push_back((float)v.imag());
        }
        while (P.pool.size() % 8) P.pool.push_back(0.f);
        add(o, 6);
        D = Diag(NA);
    }
    void emit_rots(int gate)
    {
        for (auto &r : rots) {
            DevOp o = base_op(OP_R1, gate);
            o.a = LOC_REG | r.first;
            o.mat = (int32_t)P.pool.size();
            const double *m = r.second.data();
            const float f[8] = {(float)m[0], 0.f, (float)m[1], 0.f, (float)m[2], 0.f, (float)m[3], 0.f};
            P.pool.insert(P.pool.end(), f, f + 8);
            add(o, 6);
        }
        rots.clear();
        rot_mask = 0;
    }
    // emit Dpre and the rotations as one layer op; Dpost becomes the new pending Dpre
    void flush_rots(int gate)
    {
        if (rots.empty()) {
            for (int i = 0; i < NA; ++i) pre.d[i] *= post.d[i];
            post = Diag(NA);
            return;
        }
        DevOp o = base_op(OP_LAYER, gate);
        o.mat = (int32_t)P.pool.size();
        // each rotation [[c, -s], [s, c]] is applied as three shears with
        // t = -s / (1 + c); one with c < 0 is written as -1 times the rotation
        // by the angle minus pi, and the -1 goes into the diagonal
        double ts[2 * 5] = {0};
        bool negate = false;
        uint32_t mask = 0;
        for (auto &r : rots) {
            double c = r.second[0], sn = r.second[2];
            if (c < 0) {
                c = -c;
                sn = -sn;
                negate = !negate;
            }
            ts[2 * r.first] = -sn / (1.0 + c);
            ts[2 * r.first + 1] = sn;
            mask |= 1u << r.first;
        }
        for (auto &v : pre.d) {
            const cd w = negate ? -v : v;
            P.pool.push_back((float)w.real());
            P.pool.push_back((float)w.imag());
        }
        for (int j = 0; j < R; ++j) {
            P.pool.push_back((float)ts[2 * j]);
            P.pool.push_back((float)ts[2 * j + 1]);
        }
        while (P.pool.size() % 8) P.pool.push_back(0.f);
        o.a = (int32_t)mask;
        add(o, 6.0 * rots.size() + (pre.identity() ? 0.0 : 6.0));
        rots.clear();
        rot_mask = 0;
        pre = post;
        post = Diag(NA);
    }
    // the pending fixed block (rotations and diagonals); the pending
    // parameterised diagonal commutes with it and may stay
    void flush_fixed(int gate)
    {
        flush_rots(gate);
        emit_diag(pre, gate);
    }
    void flush_all(int gate)
    {
        flush_fixed(gate);
        flush_prz();
    }
    // the pending parameterised RZ rotations as one OP_DREG: entries formed on
    // the device (ParamDiag), one gradient slot per member in slot order
    void flush_prz()
    {
        if (prz.empty()) return;
        std::sort(prz.begin(), prz.end());
        DevOp o = base_op(OP_DREG, prz[0].second);
        o.gen = GEN_Z;
        o.a = (int32_t)prz_mask;
        o.mat = (int32_t)P.pool.size();
        P.pool.insert(P.pool.end(), (size_t)2 * NA, 0.f);
        while (P.pool.size() % 8) P.pool.push_back(0.f);
        o.grad_slot = (int32_t)P.grad_param.size();
        ParamDiag pd;
        std::memset(&pd, 0, sizeof(pd));
        pd.mat = o.mat;
        pd.n = (int32_t)prz.size();
        for (size_t m = 0; m < prz.size(); ++m) {
            const int32_t th = (int32_t)(C.theta_off + P.gates[prz[m].second].param);
            pd.slot[m] = prz[m].first;
            pd.theta[m] = th;
            pd.gmat[m] = mat_of[prz[m].second];
            P.grad_param.push_back(th);
        }
        P.pdiags.push_back(pd);
        add(o, 6);
        prz.clear();
        prz_mask = 0;
    }
    // a parameterised RZ on a register slot: joins the pending diagonal
    bool is_prz(int g) const
    {
        const GateMeta &m = meta[g];
        return m.param && P.gates[g].kind == QSV_RZ && is_reg(loc(m.q[0]));
    }
    // gate g acts non-diagonally on a slot of the pending diagonal (a control
    // of CX/CU on such a slot does not)
    bool breaks_prz(int g) const
    {
        if (!prz_mask) return false;
        const GateMeta &m = meta[g];
        if (m.op == OP_D1 || m.op == OP_D2 || m.op == OP_CZ) return false;
        auto on = [&](int q) {
            const int32_t l = loc(q);
            return is_reg(l) && ((prz_mask >> (l & 0x3F)) & 1u);
        };
        if (m.op == OP_CX || m.op == OP_CU) return on(m.tgt);
        return on(m.q[0]) || (m.nq == 2 && on(m.q[1]));
    }
    // value of a gate's diagonal entry for register index i (all qubits in registers)
    cd diag_value(const GateMeta &m, int32_t la, int32_t lb, int i) const
    {
        const int ba = (i >> (la & 0x3F)) & 1;
        if (m.nq == 1) return cd(m.m[2 * (ba * 3)], m.m[2 * (ba * 3) + 1]);
        const int bb = (i >> (lb & 0x3F)) & 1;
        const int j = ba + 2 * bb;
        return cd(m.m[2 * (j * 4 + j)], m.m[2 * (j * 4 + j) + 1]);
    }
    void emit_plain(int g)
    {
        const GateMeta &m = meta[g];
        DevOp o = base_op(m.op, g);
        o.gen = m.gen;
        o.mat = mat_of[g];
        if (m.param) {
            o.grad_slot = (int32_t)P.grad_param.size();
            P.grad_param.push_back((int32_t)(C.theta_off + P.gates[g].param));
        }
        if (m.op == OP_CX || m.op == OP_CU) { o.a = loc(m.ctrl); o.b = loc(m.tgt); }
        else { o.a = loc(m.q[0]); o.b = m.nq == 2 ? loc(m.q[1]) : 0; }
        bool need_reg_a = m.op == OP_U1 || m.op == OP_R1 || m.op == OP_U2 || m.op == OP_SWAP;
        bool need_reg_b = m.op == OP_CX || m.op == OP_CU || m.op == OP_U2 || m.op == OP_SWAP;
        if ((need_reg_a && !is_reg(o.a)) || (need_reg_b && !is_reg(o.b)))
            throw std::logic_error("required qubit not in registers");
        // kinds by where the qubits are (each has its own code path in the kernel)
        if (m.op == OP_CZ) {
            if (!is_reg(o.a)) std::swap(o.a, o.b);
            if (!is_reg(o.a)) o.kind = OP_CZ_TT;
            else if (!is_reg(o.b)) o.kind = OP_CZ_RT;
        } else if (m.op == OP_CX && !is_reg(o.a)) {
            o.kind = OP_CX_T;
        } else if (m.op == OP_D1 && !is_reg(o.a)) {
            o.kind = OP_D1_T;
        } else if (m.op == OP_D2 && !(is_reg(o.a) && is_reg(o.b))) {
            if (!is_reg(o.a) && !is_reg(o.b)) {
                o.kind = OP_D2_TT;
            } else {
                o.kind = OP_D2_RT;
                if (!is_reg(o.a)) {  // the register qubit goes first: entries j = 1 and 2 trade places
                    std::swap(o.a, o.b);
                    const float *d = &P.pool[o.mat];
                    if (d[2] != d[4] || d[3] != d[5]) {
                        if (m.param) throw std::logic_error("parameterised diagonal 4x4 must be symmetric");
                        const float e[8] = {d[0], d[1], d[4], d[5], d[2], d[3], d[6], d[7]};
                        o.mat = (int32_t)P.pool.size();
                        P.pool.insert(P.pool.end(), e, e + 8);
                    }
                }
                const float *d = &P.pool[o.mat];  // entries with the register bit 0: j = 0 and 2
                if (!m.param && d[0] == 1.f && d[1] == 0.f && d[4] == 1.f && d[5] == 0.f) o.flags = 1;
            }
        }
        add(o, m.flops);
    }
    // True if folding gate g now neither closes the pending block nor emits
    // it: the condition under which gate() below only extends the block.
    bool absorbs(int g) const
    {
        const GateMeta &m = meta[g];
        if (is_prz(g)) return !((prz_mask >> (loc(m.q[0]) & 0x3F)) & 1u);
        if (breaks_prz(g)) return false;
        const bool pending = !rots.empty() || !pre.identity() || !post.identity();
        if (m.param) return !pending;
        if (m.op == OP_D1 || m.op == OP_D2 || m.op == OP_CZ) {
            const int32_t la = loc(m.q[0]), lb = m.nq == 2 ? loc(m.q[1]) : LOC_REG;
            if (is_reg(la) && is_reg(lb)) return true;
            uint32_t regs = (is_reg(la) ? 1u << (la & 0x3F) : 0u) | (m.nq == 2 && is_reg(lb) ? 1u << (lb & 0x3F) : 0u);
            return (regs & rot_mask) == 0;
        }
        if ((m.op == OP_U1 || m.op == OP_R1) && is_reg(loc(m.q[0]))) {
            const int j = loc(m.q[0]) & 0x3F;
            cd d1a, d1b, d2b;
            double c, sn;
            if (split_unitary(m.m, d1a, d1b, c, sn, d2b)) return !((rot_mask >> j) & 1u) && !post.depends_on(j);
        }
        if ((m.op == OP_CX || m.op == OP_SWAP) && is_reg(loc(m.q[0])) && is_reg(loc(m.q[1]))) return rots.empty();
        return !pending;
    }
    void gate(int g, bool fold)
    {
        const GateMeta &m = meta[g];
        if (!fold) { emit_plain(g); return; }
        const bool diag = m.op == OP_D1 || m.op == OP_D2 || m.op == OP_CZ;
        if (is_prz(g)) {
            const int j = loc(m.q[0]) & 0x3F;
            if ((prz_mask >> j) & 1u) flush_prz();   // a second one on the slot: the first goes out
            if ((rot_mask >> j) & 1u) flush_rots(g); // a pending rotation on the slot comes first
            prz.push_back({j, g});
            prz_mask |= 1u << j;
            return;
        }
        if (breaks_prz(g)) flush_prz();  // commutes with everything pending on other slots
        if (m.param) {  // matrix formed on the device: ends the fixed block
            flush_fixed(g);
            emit_plain(g);
            return;
        }
        if (diag) {
            const int32_t la = loc(m.q[0]), lb = m.nq == 2 ? loc(m.q[1]) : LOC_REG;
            const bool all_reg = is_reg(la) && is_reg(lb);
            if (all_reg) {
                for (int i = 0; i < NA; ++i) post.d[i] *= diag_value(m, la, lb, i);
                return;
            }
            // touches a thread or tile-index qubit: commutes with the block unless a pending
            // rotation acts on its register qubit
            uint32_t regs = (is_reg(la) ? 1u << (la & 0x3F) : 0u) | (m.nq == 2 && is_reg(lb) ? 1u << (lb & 0x3F) : 0u);
            if (regs & rot_mask) flush_rots(g);
            emit_plain(g);
            return;
        }
        if ((m.op == OP_U1 || m.op == OP_R1) && is_reg(loc(m.q[0]))) {
            const int j = loc(m.q[0]) & 0x3F;
            cd d1a, d1b, d2b;
            double c, sn;
            if (split_unitary(m.m, d1a, d1b, c, sn, d2b)) {
                if ((rot_mask >> j) & 1u || post.depends_on(j)) flush_rots(g);
                for (int i = 0; i < NA; ++i) {
                    if ((i >> j) & 1) {
                        pre.d[i] *= d2b;
                        post.d[i] *= d1b;
                    } else {
                        post.d[i] *= d1a;
                    }
                }
                rots.push_back({j, {c, -sn, sn, c}});
                rot_mask |= 1u << j;
                return;
            }
        }
        if ((m.op == OP_CX || m.op == OP_SWAP) && is_reg(loc(m.q[0])) && is_reg(loc(m.q[1]))) {
            // the diagonal pending before the permutation X is carried past it:
            // X D = D' X with D'(i) = D(X(i))
            flush_rots(g);
            emit_plain(g);
            Diag moved(NA);
            for (int i = 0; i < NA; ++i) {
                int k = i;
                if (m.op == OP_CX) {
                    const int c = loc(m.ctrl) & 0x3F, t = loc(m.tgt) & 0x3F;
                    if ((i >> c) & 1) k ^= 1 << t;
                } else {
                    const int a = loc(m.q[0]) & 0x3F, b = loc(m.q[1]) & 0x3F;
                    if (((i >> a) & 1) != ((i >> b) & 1)) k ^= (1 << a) | (1 << b);
                }
                moved.d[i] = pre.d[k];
            }
            pre = moved;
            return;
        }
        flush_fixed(g);
        emit_plain(g);
    }
};

// Lower a stage's gates with folding, in a dependency-respecting order chosen
// so that blocks stay open: among the gates whose predecessors (earlier gates
// on a shared qubit) are done, the first one the pending block absorbs is
// taken, else the first one.  Gates on disjoint qubits commute, so every such
// order gives the same unitary.  Returns the order used.
std::vector<int> fold_order(const std::vector<GateMeta> &meta, const std::vector<int> &gates, StageLowering &L)
{
    const int N = (int)gates.size();
    std::vector<std::vector<int>> succ(N);
    std::vector<int> npred(N, 0);
    int last[64];
    std::fill(last, last + 64, -1);
    for (int i = 0; i < N; ++i) {
        uint64_t qm = meta[gates[i]].qmask;
        std::vector<int> pr;
        while (qm) {
            const int q = __builtin_ctzll(qm);
            qm &= qm - 1;
            if (last[q] >= 0 && std::find(pr.begin(), pr.end(), last[q]) == pr.end()) pr.push_back(last[q]);
            last[q] = i;
        }
        for (int p : pr) succ[p].push_back(i);
        npred[i] = (int)pr.size();
    }
    std::set<int> ready;
    for (int i = 0; i < N; ++i)
        if (!npred[i]) ready.insert(i);
    std::vector<int> order;
    order.reserve(N);
    while (!ready.empty()) {
        int pick = *ready.begin();
        for (int i : ready)
            if (L.absorbs(gates[i])) { pick = i; break; }
        ready.erase(pick);
        L.gate(gates[pick], true);
        order.push_back(gates[pick]);
        for (int v : succ[pick])
            if (--npred[v] == 0) ready.insert(v);
    }
    return order;
}

// VALU instructions per amplitude of an op kind (for choosing a lowering).
double op_cost(int kind)
{
    switch (kind) {
    case OP_U1: return 8;
    case OP_R1: case OP_D1: case OP_D1_T: case OP_D2: case OP_D2_RT: case OP_D2_TT: case OP_DREG: return 4;
    case OP_LAYER: return 4;  // per rotation or diagonal; op_cost_of() counts them
    case OP_CU: return 9;
    case OP_U2: return 16;
    default: return 1;  // CX, CZ, SWAP: selects and moves
    }
}

}  // namespace

// Distributed level (Section 4.2 applied to the memory of one rank, Section
// 4.3's data reshaping between partitions).  2^g ranks each hold the 2^(n-g)
// amplitudes whose g highest bit positions equal the rank.  The greedy cuts
// the circuit into partitions of at most n - g local qubits; each partition
// runs with its local qubits at the low n - g positions.  Between partitions
// the qubits that become local trade positions with qubits that stop being
// local: each trade is a SWAP of a low and a high position, i.e. the
// exchange between ranks that differ in that high bit.  On one GPU the SWAPs
// run as ordinary gates; a last set of SWAPs restores the logical order.
void distribute(Plan &P, const qsv_gate *gates, int64_t G, int g)
{
    const int n = P.n, L = n - g;
    std::vector<GateMeta> meta((size_t)G);
    std::vector<int> all((size_t)G);
    for (int64_t i = 0; i < G; ++i) {
        meta[i] = classify(gates[i]);
        all[i] = (int)i;
    }
    P.dist_parts = greedy_partition(n, meta, all, L, ~0ull);
    if (P.dist_parts.empty()) P.dist_parts.push_back(Part());
    std::vector<int> pos(n), at(n);  // logical qubit -> position, position -> logical qubit
    for (int q = 0; q < n; ++q) pos[q] = at[q] = q;
    P.gates.clear();
    P.phys_logical.clear();
    P.segments.clear();
    P.remap_exchange_swaps = P.remap_swaps = 0;
    auto swap_positions = [&](int pa, int pb) {
        qsv_gate s;
        std::memset(&s, 0, sizeof(s));
        s.kind = QSV_SWAP;
        s.q0 = pa;
        s.q1 = pb;
        s.param = -1;
        P.gates.push_back(s);
        P.phys_logical.push_back(-1);
        std::swap(at[pa], at[pb]);
        pos[at[pa]] = pa;
        pos[at[pb]] = pb;
        ++P.remap_swaps;
        if ((pa < L) != (pb < L)) ++P.remap_exchange_swaps;
    };
    auto open_segment = [&](bool remap, uint64_t allowed) {
        Segment sg;
        sg.g0 = sg.g1 = (int64_t)P.gates.size();
        sg.remap = remap;
        sg.allowed = allowed;
        P.segments.push_back(sg);
    };
    auto close_segment = [&]() {
        P.segments.back().g1 = (int64_t)P.gates.size();
        if (P.segments.back().g1 == P.segments.back().g0) P.segments.pop_back();
    };
    const uint64_t low = L >= 64 ? ~0ull : (1ull << L) - 1;
    for (Part &part : P.dist_parts) {
        // pad the local set to n - g qubits with qubits that are already local (no data moves)
        uint64_t S = part.S;
        for (int p = 0; p < L && popc(S) < L; ++p) S |= 1ull << at[p];
        part.S = S;
        // remap: each qubit entering the local set (at a high position) trades
        // places with one leaving it (at a low position)
        std::vector<int> enter, leave;
        for (int p = L; p < n; ++p)
            if ((S >> at[p]) & 1) enter.push_back(p);
        for (int p = 0; p < L; ++p)
            if (!((S >> at[p]) & 1)) leave.push_back(p);
        if (enter.size() != leave.size()) throw std::logic_error("distributed local set has the wrong size");
        open_segment(true, ~0ull);
        for (size_t j = 0; j < enter.size(); ++j) swap_positions(leave[j], enter[j]);
        close_segment();
        open_segment(false, low);
        for (int gi : part.gates) {
            qsv_gate x = gates[gi];
            x.q0 = pos[x.q0];
            if (x.q1 >= 0) x.q1 = pos[x.q1];
            P.gates.push_back(x);
            P.phys_logical.push_back(gi);
        }
        close_segment();
    }
    open_segment(true, ~0ull);  // back to the logical order
    for (int p = 0; p < n; ++p)
        if (at[p] != p) swap_positions(p, pos[p]);
    close_segment();
}

void build_plan(Plan &P)
{
    const int n = P.n;
    P.meta.resize(P.gates.size());
    for (size_t i = 0; i < P.gates.size(); ++i) P.meta[i] = classify(P.gates[i]);

    // matrix pool entries, one per gate, laid out circuit by circuit: a
    // circuit's gate matrices, then the entries its lowering adds (folded
    // diagonals and layers), so that circuits of the same structure have the
    // same pool layout at different bases
    std::vector<int32_t> mat_of(P.gates.size(), -1);
    auto add_matrices = [&](int64_t g0, int64_t g1) {
        for (int64_t i = g0; i < g1; ++i) {
            const GateMeta &m = P.meta[i];
            if (m.op == OP_CX || m.op == OP_CZ || m.op == OP_SWAP) continue;
            int len = m.op == OP_U2 ? 32 : 8;
            mat_of[i] = (int32_t)P.pool.size();
            if (m.op == OP_D2) {  // diagonal entries j = b(q0) + 2 b(q1)
                for (int j = 0; j < 4; ++j) {
                    P.pool.push_back((float)m.m[2 * (j * 4 + j)]);
                    P.pool.push_back((float)m.m[2 * (j * 4 + j) + 1]);
                }
            } else {
                for (int j = 0; j < len; ++j) P.pool.push_back((float)m.m[j]);
            }
        }
    };

    P.flops = 0;
    P.bytes = 0;
    const double dim = std::ldexp(1.0, n);
    // batched plans: circuits whose gate records are identical (kinds, qubits,
    // parameter indices relative to the circuit, fixed angles and matrices)
    // share the partition, stage and op tables of the first of them; they
    // differ only in their pool base (their own rotation matrices) and their
    // gradient slots, both by a constant offset
    const bool batched = P.circ.size() > 1;
    std::unordered_map<uint64_t, std::vector<int>> by_hash;
    struct Span { int32_t pool0 = 0, pool1 = 0, slot0 = 0, slot1 = 0, pd0 = 0, pd1 = 0; double flops = 0; };
    std::vector<Span> span(P.circ.size());
    P.circ_pool_delta.assign(P.circ.size(), 0);
    P.circ_slot_delta.assign(P.circ.size(), 0);
    for (size_t ci = 0; ci < P.circ.size(); ++ci) {
        CircuitPlan &C = P.circ[ci];
        int first = -1;
        uint64_t key = 0;
        if (batched) {
            const unsigned char *b = reinterpret_cast<const unsigned char *>(P.gates.data() + C.g0);
            const size_t len = (size_t)(C.g1 - C.g0) * sizeof(qsv_gate);
            key = 1469598103934665603ull ^ len;  // FNV-1a over the gate records
            for (size_t i = 0; i < len; ++i) key = (key ^ b[i]) * 1099511628211ull;
            for (int e : by_hash[key]) {
                const CircuitPlan &E = P.circ[e];
                if (E.g1 - E.g0 == C.g1 - C.g0 &&
                    std::memcmp(P.gates.data() + E.g0, P.gates.data() + C.g0, len) == 0) {
                    first = e;
                    break;
                }
            }
        }
        span[ci].pool0 = (int32_t)P.pool.size();
        span[ci].slot0 = (int32_t)P.grad_param.size();
        span[ci].pd0 = (int32_t)P.pdiags.size();
        if (first >= 0) {  // reuse the tables of circuit `first`
            const CircuitPlan &E = P.circ[first];
            const Span &se = span[first];
            const int64_t dg = C.g0 - E.g0;
            for (int32_t i = se.pool0; i < se.pool1; ++i) P.pool.push_back(P.pool[i]);
            for (int64_t g = C.g0; g < C.g1; ++g)
                if (mat_of[g - dg] >= 0) mat_of[g] = mat_of[g - dg] - se.pool0 + span[ci].pool0;
            for (int32_t sl = se.slot0; sl < se.slot1; ++sl)
                P.grad_param.push_back((int32_t)(P.grad_param[sl] - E.theta_off + C.theta_off));
            P.circ_pool_delta[ci] = span[ci].pool0 - se.pool0;
            P.circ_slot_delta[ci] = span[ci].slot0 - se.slot0;
            for (int64_t g = C.g0; g < C.g1; ++g) {
                if (P.meta[g].param) {
                    ParamGate pg;
                    pg.mat = mat_of[g];
                    pg.kind = P.gates[g].kind;
                    pg.theta_index = (int32_t)(C.theta_off + P.gates[g].param);
                    pg.pad = 0;
                    P.pgates.push_back(pg);
                }
            }
            span[ci].pd0 = (int32_t)P.pdiags.size();
            for (int32_t d = se.pd0; d < se.pd1; ++d) {  // its folded diagonals: own pool entries and angles
                ParamDiag pd = P.pdiags[d];
                pd.mat += P.circ_pool_delta[ci];
                for (int m = 0; m < pd.n; ++m) pd.gmat[m] += P.circ_pool_delta[ci];
                for (int m = 0; m < pd.n; ++m) pd.theta[m] += (int32_t)(C.theta_off - E.theta_off);
                P.pdiags.push_back(pd);
            }
            span[ci].pd1 = (int32_t)P.pdiags.size();
            C.parts = E.parts;
            for (auto &pt : C.parts)
                for (int &g : pt.gates) g += (int)dg;
            C.stages = E.stages;
            for (auto &st : C.stages)
                for (auto &pt : st)
                    for (int &g : pt.gates) g += (int)dg;
            C.part_begin = E.part_begin;
            C.shares = first;
            span[ci].pool1 = (int32_t)P.pool.size();
            span[ci].slot1 = (int32_t)P.grad_param.size();
            span[ci].flops = se.flops;
            P.flops += se.flops;
            P.bytes += 16.0 * dim * (double)C.parts.size();
            continue;
        }
        if (batched) by_hash[key].push_back((int)ci);
        const double flops_c0 = P.flops;
        add_matrices(C.g0, C.g1);
        for (int64_t g = C.g0; g < C.g1; ++g) {
            if (P.meta[g].param) {
                ParamGate pg;
                pg.mat = mat_of[g];
                pg.kind = P.gates[g].kind;
                pg.theta_index = (int32_t)(C.theta_off + P.gates[g].param);
                pg.pad = 0;
                P.pgates.push_back(pg);
            }
        }
        std::vector<int> all;
        for (int64_t g = C.g0; g < C.g1; ++g) all.push_back((int)g);
        const int t = std::min(P.t, n);
        const int R = std::min(P.R, t);
        const int w = t - R;
        const int k = std::min(P.k, n);
        // level 1: partitions of at most k local qubits (padded to min(k, n)); a
        // distributed plan partitions each of its segments on its own
        std::vector<Segment> segs = P.segments;
        if (segs.empty()) {
            Segment whole;
            whole.g0 = C.g0;
            whole.g1 = C.g1;
            segs.push_back(whole);
        }
        for (const Segment &sg : segs) {
            std::vector<int> sub;
            for (int64_t g = sg.g0; g < sg.g1; ++g) sub.push_back((int)g);
            if (P.flags & QSV_PLAN_GATE_BY_GATE) {
                for (int g : sub) {
                    Part p;
                    p.S = P.meta[g].qmask;
                    p.gates.push_back(g);
                    C.parts.push_back(p);
                }
            } else {
                std::vector<Part> ps = greedy_partition(n, P.meta, sub, k, sg.allowed);
                C.parts.insert(C.parts.end(), ps.begin(), ps.end());
            }
        }
        if (C.parts.empty()) C.parts.push_back(Part());  // an empty circuit still gets one (empty) sweep
        C.part_begin = (int32_t)P.parts.size();
        for (auto &part : C.parts) {
            part.S = pad_low(part.S, n, std::min(k, n));
            uint64_t T = part.S;
            for (int q = 0; q < n && popc(T) < t; ++q) T |= 1ull << q;
            DevPart dp;
            std::memset(&dp, 0, sizeof(dp));
            dp.t = t;
            dp.n_glb = n - t;
            int pos_of[64];
            for (int q = 0, c = 0, b = 0; q < n; ++q) {
                if ((T >> q) & 1) { dp.tq[c] = q; pos_of[q] = c++; }
                else { dp.gq[b++] = q; pos_of[q] = -1; }
            }
            // level 2: register stages of this partition
            std::vector<Part> st = greedy_partition(n, P.meta, part.gates, R, T);
            if (st.empty()) st.push_back(Part());  // every partition has at least one stage
            dp.stage_begin = (int32_t)P.stages.size();
            for (auto &s : st) {
                DevStage ds;
                std::memset(&ds, 0, sizeof(ds));
                uint32_t posmask = 0;
                for (int q = 0; q < n; ++q)
                    if ((s.S >> q) & 1) posmask |= 1u << pos_of[q];
                stage_layout(posmask, t, R, w, ds);
                uint64_t regq = 0;
                for (int j = 0; j < R; ++j) regq |= 1ull << dp.tq[ds.regpos[j]];
                s.S = regq;
                auto loc = [&](int q) -> int32_t {
                    if (pos_of[q] < 0) return LOC_GLB | q;
                    for (int j = 0; j < R; ++j)
                        if (ds.regpos[j] == pos_of[q]) return LOC_REG | j;
                    for (int b = 0; b < w; ++b)
                        if (ds.thrpos[b] == pos_of[q]) return LOC_THR | b;
                    throw std::logic_error("qubit not in layout");
                };
                ds.op_begin = (int32_t)P.ops.size();
                // lower with diagonal folding; keep it only if it needs fewer instructions
                const size_t ops0 = P.ops.size(), pool0 = P.pool.size(), grad0 = P.grad_param.size(),
                             pd0 = P.pdiags.size();
                const double flops0 = P.flops;
                double plain_cost = 0, folded_cost = 0;
                for (int g : s.gates) plain_cost += op_cost(P.meta[g].op) + 2;  // + dispatch
                {
                    StageLowering L(P, mat_of, R, loc, C);
                    s.gates = fold_order(P.meta, s.gates, L);
                    L.flush_all(s.gates.empty() ? -1 : s.gates.back());
                    for (size_t k = ops0; k < P.ops.size(); ++k) {
                        const DevOp &o = P.ops[k];
                        // a layer op: 3 per rotation and 4 for the diagonal
                        folded_cost += (o.kind == OP_LAYER ? 3.0 * __builtin_popcount(o.a) + 4 : op_cost(o.kind)) + 2;
                    }
                }
                if (folded_cost >= plain_cost) {
                    P.ops.resize(ops0);
                    P.pool.resize(pool0);
                    P.grad_param.resize(grad0);
                    P.pdiags.resize(pd0);
                    P.flops = flops0;
                    StageLowering L(P, mat_of, R, loc, C);
                    for (int g : s.gates) L.gate(g, false);
                }
                ds.op_end = (int32_t)P.ops.size();
                P.stages.push_back(ds);
            }
            dp.stage_end = (int32_t)P.stages.size();
            C.stages.push_back(std::move(st));
            P.parts.push_back(dp);
            P.bytes += 16.0 * dim;
        }
        span[ci].pool1 = (int32_t)P.pool.size();
        span[ci].slot1 = (int32_t)P.grad_param.size();
        span[ci].pd1 = (int32_t)P.pdiags.size();
        span[ci].flops = P.flops - flops_c0;
    }
    // batched plans: longest circuits first in the work queue
    P.batch_order.resize(P.circ.size());
    for (size_t c = 0; c < P.circ.size(); ++c) P.batch_order[c] = (int32_t)c;
    std::stable_sort(P.batch_order.begin(), P.batch_order.end(), [&](int32_t x, int32_t y) {
        return P.circ[x].g1 - P.circ[x].g0 > P.circ[y].g1 - P.circ[y].g0;
    });
    // theta index -> gradient slots, in slot order (deterministic sums)
    P.param_off.assign(P.n_params + 1, 0);
    for (int32_t p : P.grad_param) P.param_off[p + 1]++;
    for (int64_t i = 0; i < P.n_params; ++i) P.param_off[i + 1] += P.param_off[i];
    P.param_slots.assign(P.grad_param.size(), 0);
    std::vector<int32_t> fill(P.param_off.begin(), P.param_off.end() - (P.n_params >= 0 ? 1 : 0));
    for (size_t s = 0; s < P.grad_param.size(); ++s) P.param_slots[fill[P.grad_param[s]]++] = (int32_t)s;
}

}  // namespace qsv
