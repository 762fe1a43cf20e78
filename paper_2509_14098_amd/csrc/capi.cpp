// C interface (include/qsv.h).  Argument checking, plan construction and
// upload, and the launch sequences of qsv_apply / qsv_expect /
// qsv_adjoint_grad.  No C++ exception crosses the interface.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <atomic>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"

using namespace qsv;

namespace {

thread_local std::string g_err;

// Largest states: 2^35 complex64 amplitudes (256 GiB) is the largest power of
// two that fits one MI355X's 288 GB of HBM; host-only plans (no device
// tables) reach the qubit counts of multi-GPU runs, e.g. the 40-qubit circuit
// whose 32-qubit rank share the sweeps run on.
constexpr int MAX_DEVICE_QUBITS = 35;
constexpr int MAX_HOST_QUBITS = 40;

struct Fail {
    qsv_status code;
    std::string msg;
};

[[noreturn]] void fail(qsv_status code, const std::string &msg) { throw Fail{code, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(QSV_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
qsv_status guarded(F &&f)
{
    try {
        f();
        g_err.clear();
        return QSV_OK;
    } catch (const Fail &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return QSV_E_NOMEM;
    } catch (const std::exception &e) {
        g_err = std::string("internal error: ") + e.what();
        return QSV_E_ARG;
    }
}

template <typename T>
T *dev_upload(const std::vector<T> &v)
{
    if (v.empty()) return nullptr;
    void *p = nullptr;
    if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) fail(QSV_E_NOMEM, "device allocation failed");
    hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    return static_cast<T *>(p);
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

// Smallest supported kernel shape that covers n qubits when the state fits
// one tile; otherwise the configured shape.
void choose_shape(int n, int R, int LW, int &Re, int &LWe, int &te)
{
    if (n >= R + LW) {
        Re = R; LWe = LW; te = R + LW;
        return;
    }
    te = n;
    for (int r = std::min(R, n); r <= std::min(5, n); ++r) {
        int w = n - r;
        for (int lw : {6, 8, 9, 10}) {
            if (lw >= w && kernel_shape_supported(r, lw)) {
                Re = r; LWe = lw;
                return;
            }
        }
    }
    fail(QSV_E_UNSUPPORTED, "no kernel shape for this qubit count");
}

}  // namespace

// ---------------------------------------------------------------------------
struct qsv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool timing = false;
    double last_ms = 0;
    int64_t last_launches = 0;
    std::vector<hipEvent_t> events;
    // scratch
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *lam = nullptr;
    size_t lam_bytes = 0;
    void *terms_dev = nullptr;
    size_t terms_bytes = 0;
    // qsv_expect: the tables of the last sum, kept on the device while the
    // same terms come again (key: n and the term records)
    void *expect_dev = nullptr;
    size_t expect_bytes = 0;
    std::string expect_key;
    DevPass *expect_dp = nullptr;
    DevGroup *expect_dg = nullptr;
    DevTerm *expect_dt = nullptr;
    int expect_np = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t pinned_ready = nullptr;
    hipEvent_t handoff = nullptr;  // orders work across a change of stream
    hipEvent_t pace[2] = {nullptr, nullptr};  // qsv_apply's sweeps in flight while a compile is pending
    // qsv_expect_noalloc: pinned staging of the grouped terms, allocated once by qsv_create
    void *na_staging = nullptr;
    hipEvent_t na_staging_ready = nullptr;
    int *queue = nullptr;
    int n_cu = 0;

    // batched launches with timing on: per workgroup its start and exit on the
    // device's real-time clock
    uint64_t *wg_clock = nullptr;
    int wg_clock_n = 0;   // workgroups of the last timed batched launch
    uint64_t *batch_clock(int grid)
    {
        if (!timing) {
            wg_clock_n = 0;
            return nullptr;
        }
        if (!wg_clock && hipMalloc((void **)&wg_clock, sizeof(uint64_t) * 2 * 4096) != hipSuccess)
            fail(QSV_E_NOMEM, "clock buffer allocation failed");
        wg_clock_n = std::min(grid, 4096);
        return grid <= 4096 ? wg_clock : nullptr;
    }
    int *ensure_queue()
    {
        if (!queue && hipMalloc((void **)&queue, 256) != hipSuccess) fail(QSV_E_NOMEM, "queue allocation failed");
        return queue;
    }
    int grid_batched(int n_items)
    {
        if (n_cu == 0) hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device), "attr");
        return std::max(1, std::min(n_cu, n_items));
    }

    void *ensure(void *&p, size_t &have, size_t need)
    {
        if (need > have) {
            if (p) {
                hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
                dev_free(p);
                p = nullptr;
                have = 0;
            }
            if (hipMalloc(&p, need) != hipSuccess) fail(QSV_E_NOMEM, "device scratch allocation failed");
            have = need;
        }
        return p;
    }
};

struct qsv_plan : public Plan {};

// A term in the kernels' form: coeff * i^{#Y} as (re, im), and its Z/Y mask.
static DevTerm dev_term(const qsv_pauli_term &h)
{
    const int ny = __builtin_popcountll(h.x_mask & h.z_mask) & 3;  // i^{#Y}
    const double c = h.coeff;
    DevTerm d;
    d.cre = ny == 0 ? c : ny == 2 ? -c : 0.0;
    d.cim = ny == 1 ? c : ny == 3 ? -c : 0.0;
    d.z_mask = h.z_mask;
    d.zt = 0;
    d.slot = 0;
    return d;
}

// Checks a Pauli sum against n qubits.
static void check_terms(const qsv_pauli_term *H, int n_terms, int n)
{
    if (n_terms < 0 || (n_terms > 0 && !H)) fail(QSV_E_ARG, "null or negative Pauli sum");
    const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (int t = 0; t < n_terms; ++t)
        if ((H[t].x_mask & ~full) || (H[t].z_mask & ~full)) fail(QSV_E_ARG, "Pauli mask beyond n_qubits");
}

// Groups the terms by X mask: groups in increasing mask order, terms in input
// order inside a group.  idx (n_terms entries) is scratch; groups and terms
// receive at most n_terms records each.  Returns the number of groups.
// Allocates nothing.
static int group_into(const qsv_pauli_term *H, int n_terms, int *idx, DevGroup *groups, DevTerm *terms)
{
    for (int t = 0; t < n_terms; ++t) idx[t] = t;
    std::sort(idx, idx + n_terms, [&](int a, int b) {
        return H[a].x_mask != H[b].x_mask ? H[a].x_mask < H[b].x_mask : a < b;
    });
    int g = -1;
    for (int i = 0; i < n_terms; ++i) {
        const qsv_pauli_term &h = H[idx[i]];
        if (g < 0 || h.x_mask != groups[g].x_mask) {
            ++g;
            groups[g].x_mask = h.x_mask;
            groups[g].term_begin = i;
            groups[g].xt = 0;
            groups[g].pad = 0;
        }
        groups[g].term_end = i + 1;
        terms[i] = dev_term(h);
    }
    return g + 1;
}

struct HostGroups {
    std::vector<DevPass> passes;  // expectation passes (qsv_expect only)
    std::vector<DevGroup> groups;
    std::vector<DevTerm> terms;
};

static HostGroups group_terms(const qsv_pauli_term *H, int n_terms, int n, bool passes)
{
    check_terms(H, n_terms, n);
    HostGroups g;
    std::vector<int> idx(n_terms);
    g.groups.resize(n_terms);
    g.terms.resize(n_terms);
    g.groups.resize(group_into(H, n_terms, idx.data(), g.groups.data(), g.terms.data()));
    if (passes) {
        g.passes.resize(g.groups.size());
        g.passes.resize(
            plan_expect_passes(n, g.groups.data(), (int)g.groups.size(), g.terms.data(), g.passes.data()));
    }
    return g;
}

// Byte offsets of passes, groups and terms in one upload.
struct TermLayout {
    size_t groups = 0, terms = 0, end = 0;
};
static TermLayout term_layout(size_t n_passes, size_t n_groups, size_t n_terms)
{
    auto up = [](size_t x) { return (x + 15) & ~size_t(15); };
    TermLayout L;
    L.groups = up(n_passes * sizeof(DevPass));
    L.terms = L.groups + up(n_groups * sizeof(DevGroup));
    L.end = L.terms + n_terms * sizeof(DevTerm);
    return L;
}

// Upload grouped terms (and passes) into a device buffer of the context
// (pinned staging + async copy): terms_dev unless another is given.
static void upload_groups(qsv_ctx *ctx, const HostGroups &g, DevPass *&dpasses, DevGroup *&dgroups, DevTerm *&dterms,
                          void **buf = nullptr, size_t *buf_bytes = nullptr)
{
    const TermLayout L = term_layout(g.passes.size(), g.groups.size(), g.terms.size());
    const size_t need = L.end + 64;
    if (ctx->pinned_ready) hip_check(hipEventSynchronize(ctx->pinned_ready), "hipEventSynchronize");
    if (need > ctx->pinned_bytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        if (hipHostMalloc(&ctx->pinned, need) != hipSuccess) fail(QSV_E_NOMEM, "pinned allocation failed");
        ctx->pinned_bytes = need;
    }
    char *dev = buf ? (char *)ctx->ensure(*buf, *buf_bytes, need) : (char *)ctx->ensure(ctx->terms_dev, ctx->terms_bytes, need);
    char *h = (char *)ctx->pinned;
    if (!g.passes.empty()) std::memcpy(h, g.passes.data(), g.passes.size() * sizeof(DevPass));
    if (!g.groups.empty()) std::memcpy(h + L.groups, g.groups.data(), g.groups.size() * sizeof(DevGroup));
    if (!g.terms.empty()) std::memcpy(h + L.terms, g.terms.data(), g.terms.size() * sizeof(DevTerm));
    hip_check(hipMemcpyAsync(dev, h, L.end, hipMemcpyHostToDevice, ctx->stream), "hipMemcpyAsync");
    if (!ctx->pinned_ready) hip_check(hipEventCreateWithFlags(&ctx->pinned_ready, hipEventDisableTiming), "event");
    hip_check(hipEventRecord(ctx->pinned_ready, ctx->stream), "hipEventRecord");
    dpasses = g.passes.empty() ? nullptr : (DevPass *)dev;
    dgroups = g.groups.empty() ? nullptr : (DevGroup *)(dev + L.groups);
    dterms = g.terms.empty() ? nullptr : (DevTerm *)(dev + L.terms);
}

extern "C" {

const char *qsv_last_error(void) { return g_err.c_str(); }

qsv_status qsv_create(int32_t device, void *hip_stream, qsv_ctx **out)
{
    return guarded([&] {
        if (!out) fail(QSV_E_ARG, "out is null");
        int count = 0;
        hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (device < 0 || device >= count) fail(QSV_E_DEVICE, "no such device");
        hip_check(hipSetDevice(device), "hipSetDevice");
        // set-up of qsv_expect_noalloc: the device address of its static scratch
        // (once per device) and this context's pinned staging buffer
        hip_check(noalloc_scratch_init(device), "hipGetSymbolAddress(scratch)");
        void *staging = nullptr;
        if (hipHostMalloc(&staging, NOALLOC_TERMS_BYTES) != hipSuccess) fail(QSV_E_NOMEM, "pinned allocation failed");
        hipEvent_t ready = nullptr;
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(staging);
            fail(QSV_E_DEVICE, "hipEventCreate failed");
        }
        qsv_ctx *c = new qsv_ctx();
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        c->na_staging = staging;
        c->na_staging_ready = ready;
        *out = c;
    });
}

qsv_status qsv_destroy(qsv_ctx *ctx)
{
    return guarded([&] {
        if (!ctx) return;
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        dev_free(ctx->scratch);
        dev_free(ctx->lam);
        dev_free(ctx->terms_dev);
        dev_free(ctx->expect_dev);
        dev_free(ctx->queue);
        dev_free(ctx->wg_clock);
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        if (ctx->pinned_ready) (void)hipEventDestroy(ctx->pinned_ready);
        if (ctx->handoff) (void)hipEventDestroy(ctx->handoff);
        for (hipEvent_t e : ctx->pace)
            if (e) (void)hipEventDestroy(e);
        if (ctx->na_staging) (void)hipHostFree(ctx->na_staging);
        if (ctx->na_staging_ready) (void)hipEventDestroy(ctx->na_staging_ready);
        for (auto e : ctx->events) (void)hipEventDestroy(e);
        delete ctx;
    });
}

qsv_status qsv_set_stream(qsv_ctx *ctx, void *hip_stream)
{
    return guarded([&] {
        if (!ctx) fail(QSV_E_ARG, "ctx is null");
        hipStream_t next = (hipStream_t)hip_stream;
        if (next == ctx->stream) return;
        // the context's scratch buffers are shared by every call: work queued on the new
        // stream waits for what the old stream still has in flight
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        if (!ctx->handoff) hip_check(hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventRecord(ctx->handoff, ctx->stream), "hipEventRecord");
        hip_check(hipStreamWaitEvent(next, ctx->handoff, 0), "hipStreamWaitEvent");
        ctx->stream = next;
    });
}

qsv_status qsv_set_timing(qsv_ctx *ctx, int32_t enable)
{
    return guarded([&] {
        if (!ctx) fail(QSV_E_ARG, "ctx is null");
        ctx->timing = enable != 0;
    });
}

qsv_status qsv_last_sweep_ms(qsv_ctx *ctx, double *total_ms, int64_t *n_launches)
{
    return guarded([&] {
        if (!ctx || !total_ms || !n_launches) fail(QSV_E_ARG, "null argument");
        if (ctx->timing && !ctx->events.empty() && ctx->last_launches > 0) {
            hip_check(hipEventSynchronize(ctx->events[2 * ctx->last_launches - 1]), "hipEventSynchronize");
            double total = 0;
            for (int64_t i = 0; i < ctx->last_launches; ++i) {
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]), "hipEventElapsedTime");
                total += ms;
            }
            ctx->last_ms = total;
        }
        *total_ms = ctx->last_ms;
        *n_launches = ctx->last_launches;
    });
}

qsv_status qsv_last_batch_clock(qsv_ctx *ctx, uint64_t *ticks_out, int64_t cap, int64_t *n_workgroups,
                                double *ticks_per_s)
{
    return guarded([&] {
        if (!ctx || !n_workgroups || cap < 0 || (cap > 0 && !ticks_out)) fail(QSV_E_ARG, "null argument");
        *n_workgroups = ctx->wg_clock_n;
        if (ticks_per_s) {
            int hz = 0;  // kHz
            hip_check(hipDeviceGetAttribute(&hz, hipDeviceAttributeWallClockRate, ctx->device), "attr");
            *ticks_per_s = 1e3 * hz;
        }
        if (ctx->wg_clock_n > 0 && cap > 0) {
            hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
            const int64_t n = std::min<int64_t>(cap, 2 * (int64_t)ctx->wg_clock_n);
            hip_check(hipMemcpy(ticks_out, ctx->wg_clock, sizeof(uint64_t) * n, hipMemcpyDeviceToHost), "hipMemcpy");
        }
    });
}

qsv_status qsv_last_sweep_times(qsv_ctx *ctx, float *ms_out, int64_t cap, int64_t *n_launches)
{
    return guarded([&] {
        if (!ctx || !n_launches || cap < 0 || (cap > 0 && !ms_out)) fail(QSV_E_ARG, "null argument");
        *n_launches = ctx->timing ? ctx->last_launches : 0;
        if (*n_launches > 0) {
            hip_check(hipEventSynchronize(ctx->events[2 * ctx->last_launches - 1]), "hipEventSynchronize");
            for (int64_t i = 0; i < std::min(cap, *n_launches); ++i)
                hip_check(hipEventElapsedTime(&ms_out[i], ctx->events[2 * i], ctx->events[2 * i + 1]),
                          "hipEventElapsedTime");
        }
    });
}

// Build (and, with a context, upload) a plan for validated input.
static qsv_plan *make_plan(qsv_ctx *ctx, int n_qubits, const qsv_gate *gates, const std::vector<int64_t> &off,
                           uint32_t flags, int k, int R, int LW, int n_global = 0)
{
    const int n_circuits = (int)off.size() - 1;
    auto P = new qsv_plan();
    std::unique_ptr<qsv_plan, void (*)(qsv_plan *)> guard(P, [](qsv_plan *p) { qsv_plan_destroy(p); });
    P->n = n_qubits;
    P->n_circuits = n_circuits;
    P->flags = flags;
    // a register stage must hold every gate's required qubits (up to 2)
    int need_r = 1;
    for (int64_t g = 0; g < off[n_circuits]; ++g) need_r = std::max(need_r, __builtin_popcountll(classify(gates[g]).req));
    if (n_circuits > 1) {
        P->R = R;
        P->LW = LW;
        P->t = n_qubits;
    } else {
        choose_shape(n_qubits, std::max(R, std::min(need_r, n_qubits)), LW, P->R, P->LW, P->t);
    }
    P->k = std::min(k, n_qubits);
    std::vector<int64_t> offs = off;
    if (n_global > 0) {  // one circuit: its physical gate list (relabelled, with remap SWAPs)
        P->n_global = n_global;
        distribute(*P, gates, off[1], n_global);
        offs = {0, (int64_t)P->gates.size()};
    } else {
        P->gates.assign(gates, gates + off[n_circuits]);
    }
    int64_t theta_off = 0;
    for (int c = 0; c < n_circuits; ++c) {
        CircuitPlan C;
        C.g0 = offs[c];
        C.g1 = offs[c + 1];
        int64_t np = 0;
        for (int64_t g = C.g0; g < C.g1; ++g) np = std::max<int64_t>(np, (int64_t)P->gates[g].param + 1);
        C.theta_off = theta_off;
        C.n_params = np;
        theta_off += np;
        P->circ.push_back(C);
    }
    P->n_params = theta_off;
    build_plan(*P);
    if (ctx) {
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        P->device = ctx->device;
        P->d_ops = dev_upload(P->ops);
        P->d_stages = dev_upload(P->stages);
        P->d_parts = dev_upload(P->parts);
        std::vector<float> pool = P->pool;
        pool.resize(pool.size() + 8, 0.f);  // op prefetch reads 8 floats at any offset
        P->d_pool = dev_upload(pool);
        P->d_pgates = dev_upload(P->pgates);
        P->d_pdiags = dev_upload(P->pdiags);
        P->d_grad_param = dev_upload(P->grad_param);
        P->d_param_off = dev_upload(P->param_off);
        P->d_param_slots = dev_upload(P->param_slots);
        if (n_circuits > 1) {
            std::vector<int32_t> cpart;
            std::vector<int64_t> ctheta, cnpar;
            for (auto &C : P->circ) {
                cpart.push_back(C.part_begin);
                ctheta.push_back(C.theta_off);
                cnpar.push_back(C.n_params);
            }
            P->d_batch_order = dev_upload(P->batch_order);
            P->d_circ_part = dev_upload(cpart);
            P->d_circ_theta = dev_upload(ctheta);
            P->d_circ_npar = dev_upload(cnpar);
            P->d_circ_pool_delta = dev_upload(P->circ_pool_delta);
            P->d_circ_slot_delta = dev_upload(P->circ_slot_delta);
        }
    }
    return guard.release();
}

// ---------------------------------------------------------------------------
// Autotuner: time the whole circuit for each candidate (k, tile shape) on a
// scratch state of the real size and keep the fastest.  Results are cached per
// (device, qubit count, flags, gate bytes) for the life of the process.
struct TuneChoice {
    int k, R, LW;
    double ms;
};
static std::map<std::pair<int, size_t>, TuneChoice> g_tune_cache;
static std::vector<TuneChoice> g_last_tune;
static std::mutex g_tune_mutex;  // the cache and the last-run record are process-wide

// Loads compiled programs of specialised kernels into the plan (current
// device): the forward kernel of every partition the chunks cover and, with
// rev, its reverse kernel.
static void load_spec(Plan &plan, const std::vector<SpecChunk> &chunks, bool rev)
{
    std::vector<void *> fn(plan.parts.size(), nullptr), rfn(rev ? plan.parts.size() : 0, nullptr), mods;
    std::string lerr;
    for (const SpecChunk &c : chunks) {
        hipModule_t m = nullptr;
        if (hipModuleLoadData(&m, c.code.data()) != hipSuccess) {
            lerr = "hipModuleLoadData failed";
            break;
        }
        mods.push_back((void *)m);
        for (int p = c.p0; p < c.p1 && lerr.empty(); ++p) {
            for (int r = 0; r < (rev ? 2 : 1) && lerr.empty(); ++r) {
                hipFunction_t f = nullptr;
                const std::string name = (r ? "qsv_rspec_" : "qsv_spec_") + std::to_string(p);
                if (hipModuleGetFunction(&f, m, name.c_str()) != hipSuccess) lerr = "hipModuleGetFunction " + name;
                (r ? rfn : fn)[p] = (void *)f;
            }
        }
        if (!lerr.empty()) break;
    }
    if (!lerr.empty()) {
        (void)hipGetLastError();
        for (void *m : mods) (void)hipModuleUnload((hipModule_t)m);
        fail(QSV_E_DEVICE, lerr);
    }
    for (void *m : plan.spec_modules) (void)hipModuleUnload((hipModule_t)m);
    plan.spec_fn = std::move(fn);
    plan.spec_rev_fn = std::move(rfn);
    plan.spec_modules = std::move(mods);
}

}  // extern "C"

// A compile of a plan's specialised kernels running on a host thread of its own
// (the compiler itself runs in helper processes), program by program.  The thread only reads the plan and publishes each finished
// program; the programs are loaded, and the plan changed, on the caller's
// thread.
struct qsv::AsyncSpecialise {
    std::thread worker;
    std::atomic<bool> done{false};
    std::atomic<bool> sized{false};               // chunks and ready are sized
    std::vector<SpecChunk> chunks;
    std::unique_ptr<std::atomic<bool>[]> ready;   // program c's code object is in chunks[c]
    std::vector<char> loaded;                     // caller's thread only
    size_t n_loaded = 0;
    bool rev = false;
    std::string err;
    std::chrono::steady_clock::time_point t0, t1;  // compile started, compile over (worker thread)
};

extern "C" {

// Loads one program of specialised kernels into the plan (current device):
// the forward and, with rev, the reverse kernel of each of its partitions.
static void load_chunk(Plan &plan, const SpecChunk &c, bool rev)
{
    hipModule_t m = nullptr;
    if (hipModuleLoadData(&m, c.code.data()) != hipSuccess) {
        (void)hipGetLastError();
        fail(QSV_E_DEVICE, "hipModuleLoadData failed");
    }
    std::vector<void *> fn, rfn;
    for (int p = c.p0; p < c.p1; ++p)
        for (int r = 0; r < (rev ? 2 : 1); ++r) {
            hipFunction_t f = nullptr;
            const std::string name = (r ? "qsv_rspec_" : "qsv_spec_") + std::to_string(p);
            if (hipModuleGetFunction(&f, m, name.c_str()) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipModuleUnload(m);
                fail(QSV_E_DEVICE, "hipModuleGetFunction " + name);
            }
            (r ? rfn : fn).push_back((void *)f);
        }
    plan.spec_modules.push_back((void *)m);
    for (int p = c.p0; p < c.p1; ++p) {
        plan.spec_fn[p] = fn[p - c.p0];
        if (rev) plan.spec_rev_fn[p] = rfn[p - c.p0];
    }
}

// Loads the specialised batched kernel qsv_bspec from its code object.
static void load_batched(Plan &plan, const std::vector<char> &code)
{
    hipModule_t m = nullptr;
    if (hipModuleLoadData(&m, code.data()) != hipSuccess) {
        (void)hipGetLastError();
        fail(QSV_E_DEVICE, "hipModuleLoadData failed");
    }
    hipFunction_t f = nullptr;
    if (hipModuleGetFunction(&f, m, "qsv_bspec") != hipSuccess) {
        (void)hipGetLastError();
        (void)hipModuleUnload(m);
        fail(QSV_E_DEVICE, "hipModuleGetFunction qsv_bspec");
    }
    plan.spec_modules.push_back((void *)m);
    plan.spec_batch_fn = (void *)f;
}

// Takes up what a background compile of `plan` has finished: loads every
// program that is ready (its partitions launch their specialised kernels from
// then on); with wait, first waits for the whole compile.  When the compile is
// over the plan is marked specialised (or, if it failed, keeps the programs
// loaded so far and the error for qsv_plan_specialise).  Returns whether a
// compile is still pending.
static bool finish_async(Plan &plan, bool wait)
{
    if (!plan.async_spec) return false;
    AsyncSpecialise &a = *plan.async_spec;
    if (wait && a.worker.joinable()) a.worker.join();
    const bool done = a.done.load(std::memory_order_acquire);
    if (a.sized.load(std::memory_order_acquire)) {
        const size_t n = a.chunks.size();
        if (a.loaded.size() != n) {
            a.loaded.assign(n, 0);
            plan.spec_fn.assign(plan.parts.size(), nullptr);
            plan.spec_rev_fn.assign(a.rev ? plan.parts.size() : 0, nullptr);
        }
        for (size_t c = 0; c < n; ++c)
            if (!a.loaded[c] && a.ready[c].load(std::memory_order_acquire)) {
                if (plan.n_circuits > 1)
                    load_batched(plan, a.chunks[c].code);
                else
                    load_chunk(plan, a.chunks[c], a.rev);
                a.loaded[c] = 1;
                ++a.n_loaded;
            }
    }
    if (!done) return true;
    if (a.worker.joinable()) a.worker.join();
    std::shared_ptr<AsyncSpecialise> keep = std::move(plan.async_spec);
    if (!a.err.empty() || a.n_loaded != a.chunks.size()) {
        plan.specialise_error = a.err.empty() ? "background compile incomplete" : a.err;
        return false;
    }
    plan.specialised = true;
    plan.specialise_seconds = std::chrono::duration<double>(a.t1 - a.t0).count();  // the compile's own time
    return false;
}

static TuneChoice autotune(qsv_ctx *ctx, int n, const qsv_gate *gates, const std::vector<int64_t> &off, uint32_t flags,
                           int k_fixed)
{
    const bool spec = flags & QSV_PLAN_TUNE_SPECIALISED;
    flags &= ~QSV_PLAN_TUNE_SPECIALISED;
    std::string key((const char *)gates, sizeof(qsv_gate) * (size_t)off.back());
    key += std::to_string(n) + "/" + std::to_string(flags) + "/" + std::to_string(k_fixed) + (spec ? "/s" : "");
    auto ck = std::make_pair(ctx->device, std::hash<std::string>()(key));
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(ck);
    if (it != g_tune_cache.end()) return it->second;
    TuneChoice best{k_fixed ? k_fixed : std::min(9, n), 4, 8, -1.0};
    g_last_tune.clear();
    void *psi = nullptr;
    if (hipMalloc(&psi, (size_t)8 << n) != hipSuccess) {
        (void)hipGetLastError();
        return best;  // no room for a trial state: default shape
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Release {  // also on an error thrown by a candidate
        qsv_ctx *ctx;
        void *&psi;
        hipEvent_t &e0, &e1;
        ~Release()
        {
            (void)hipStreamSynchronize(ctx->stream);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            dev_free(psi);
        }
    } release{ctx, psi, e0, e1};
    hip_check(hipMemsetAsync(psi, 0, (size_t)8 << n, ctx->stream), "hipMemsetAsync");
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    // (3, 8): 11-qubit tiles, twice the workgroups of (4, 8) for states of ~20 qubits
    const int shapes[][2] = {{5, 8}, {4, 8}, {4, 9}, {5, 9}, {4, 10}, {3, 8}, {3, 9}, {3, 10}};
    for (auto &sh : shapes) {
        const int R = sh[0], LW = sh[1], t = R + LW;
        if ((flags & QSV_PLAN_GRAD) && t > 13) continue;
        if (spec && t > 13) continue;  // specialised sweeps take tiles of at most 13 qubits
        for (int k : {8, 10, 12}) {
            if (k_fixed) k = k_fixed;
            if (k >= t || k > n) {
                if (k_fixed) break;
                continue;
            }
            qsv_plan *P = make_plan(ctx, n, gates, off, flags, k, R, LW);
            std::unique_ptr<qsv_plan, void (*)(qsv_plan *)> guard(P, [](qsv_plan *p) { qsv_plan_destroy(p); });
            // time an evenly spaced sample of at most 8 partition sweeps (after one warm-up
            // sweep) and scale it to the whole circuit
            const int np = (int)P->parts.size(), ns = std::min(np, 8);
            std::vector<int> sample;
            for (int i = 0; i < ns; ++i) sample.push_back((int)(((int64_t)2 * i + 1) * np / (2 * ns)));
            if (spec) {  // the sampled partitions as specialised kernels
                std::vector<SpecChunk> chunks;
                const std::string err = specialise_compile(*P, chunks, 16, &sample);
                if (!err.empty()) fail(QSV_E_DEVICE, err);
                load_spec(*P, chunks, false);
            }
            float ms = 0;
            hip_check(launch_sweep(*P, P->R, P->LW, sample[0], (float2 *)psi, nullptr, ctx->stream), "sweep");
            hip_check(hipEventRecord(e0, ctx->stream), "hipEventRecord");
            for (int p : sample)
                hip_check(launch_sweep(*P, P->R, P->LW, p, (float2 *)psi, nullptr, ctx->stream), "sweep");
            hip_check(hipEventRecord(e1, ctx->stream), "hipEventRecord");
            hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
            hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            ms *= (float)np / (float)ns;
            g_last_tune.push_back(TuneChoice{k, R, LW, ms});
            if (best.ms < 0 || ms < best.ms) best = TuneChoice{k, R, LW, ms};
            if (k_fixed) break;
        }
    }
    g_tune_cache[ck] = best;
    return best;
}

qsv_status qsv_partition(qsv_ctx *ctx, int32_t n_qubits, const qsv_gate *gates, const int64_t *circ_offsets,
                         int32_t n_circuits, int32_t k_local, uint32_t flags, const qsv_tile_config *tile,
                         qsv_plan **out)
{
    return guarded([&] {
        auto t0 = std::chrono::steady_clock::now();
        if (!out) fail(QSV_E_ARG, "out is null");
        if (n_qubits < 1 || n_qubits > (ctx ? MAX_DEVICE_QUBITS : MAX_HOST_QUBITS))
            fail(QSV_E_ARG, ctx ? "n_qubits must be in [1, 35]" : "n_qubits must be in [1, 40] for a host-only plan");
        if (k_local < 0) fail(QSV_E_ARG, "k_local must be >= 0");
        if (n_circuits < 1) fail(QSV_E_ARG, "n_circuits must be >= 1");
        if (flags & ~(QSV_PLAN_GATE_BY_GATE | QSV_PLAN_GRAD | QSV_PLAN_TUNE_SPECIALISED)) fail(QSV_E_ARG, "unknown flag");
        if (!circ_offsets) fail(QSV_E_ARG, "circ_offsets is null");
        std::vector<int64_t> off(n_circuits + 1, 0);
        for (int c = 0; c <= n_circuits; ++c) off[c] = circ_offsets[c];
        if (off[0] != 0) fail(QSV_E_ARG, "circ_offsets[0] must be 0");
        for (int c = 0; c < n_circuits; ++c)
            if (off[c + 1] < off[c]) fail(QSV_E_ARG, "circ_offsets must be non-decreasing");
        const int64_t G = off[n_circuits];
        if (G > 0 && !gates) fail(QSV_E_ARG, "gates is null");
        if (n_circuits > 1 && n_qubits > 14) fail(QSV_E_ARG, "batched plans need n_qubits <= 14");
        for (int c = 0; c < n_circuits; ++c)
            for (int64_t g = off[c]; g < off[c + 1]; ++g) {
                std::string e = validate_gate(gates[g], n_qubits, 0);
                if (!e.empty()) {
                    bool range = e.find("param") != std::string::npos;
                    fail(range ? QSV_E_RANGE : QSV_E_ARG, "gate " + std::to_string(g - off[c]) + ": " + e);
                }
            }
        bool user_tile = tile && (tile->reg_qubits || tile->log_threads);
        int R = 4, LW = 8;  // default shape: 4 register qubits, 256 threads, 12-qubit tiles
        if (user_tile) {
            R = tile->reg_qubits;
            LW = tile->log_threads;
            if (!kernel_shape_supported(R, LW)) fail(QSV_E_ARG, "unsupported tile shape");
        }
        if (n_circuits > 1) {
            if (n_qubits < 4) fail(QSV_E_UNSUPPORTED, "batched plans need n_qubits >= 4");
            R = 4;  // the batched kernel's shape: 4 register qubits x 1024 threads
            LW = 10;
        }
        if ((flags & QSV_PLAN_GRAD) && n_circuits == 1 && R + LW > 13 && n_qubits > 13)
            fail(QSV_E_UNSUPPORTED, "gradient plans need a tile of at most 13 qubits");
        int k = k_local == 0 ? (n_qubits <= R + LW ? n_qubits : R + LW - 3) : k_local;
        if (n_circuits > 1) k = n_qubits;  // one partition per circuit: the whole state stays on chip
        const bool tune_spec = flags & QSV_PLAN_TUNE_SPECIALISED;
        flags &= ~QSV_PLAN_TUNE_SPECIALISED;
        if ((k_local == 0 || tune_spec) && ctx && n_circuits == 1 && !user_tile && n_qubits > R + LW &&
            !(flags & QSV_PLAN_GATE_BY_GATE)) {
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            TuneChoice c = autotune(ctx, n_qubits, gates, off, flags | (tune_spec ? QSV_PLAN_TUNE_SPECIALISED : 0u),
                                    k_local);
            k = c.k;
            R = c.R;
            LW = c.LW;
        }
        if (n_qubits > R + LW && k >= R + LW) fail(QSV_E_ARG, "k_local must be below the tile size");
        qsv_plan *P = make_plan(ctx, n_qubits, gates, off, flags, k, R, LW);
        P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P;
    });
}

// Candidates timed by the last autotuning run of this process: (k, R, LW, ms) x n.
int32_t qsv_last_autotune(int32_t *out, int32_t cap)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    int32_t n = (int32_t)g_last_tune.size();
    for (int32_t i = 0; out && i < std::min(n, cap); ++i) {
        out[4 * i] = g_last_tune[i].k;
        out[4 * i + 1] = g_last_tune[i].R;
        out[4 * i + 2] = g_last_tune[i].LW;
        out[4 * i + 3] = (int32_t)(g_last_tune[i].ms * 1000.0);
    }
    return n;
}

qsv_status qsv_plan_destroy(qsv_plan *plan)
{
    return guarded([&] {
        if (!plan) return;
        if (plan->async_spec) plan->async_spec->worker.join();  // its compile is discarded
        if (plan->device >= 0) (void)hipSetDevice(plan->device);
        dev_free(plan->d_ops);
        dev_free(plan->d_stages);
        dev_free(plan->d_parts);
        dev_free(plan->d_pool);
        dev_free(plan->d_pgates);
        dev_free(plan->d_pdiags);
        dev_free(plan->d_grad_param);
        dev_free(plan->d_param_off);
        dev_free(plan->d_param_slots);
        dev_free(plan->d_batch_order);
        dev_free(plan->d_circ_part);
        dev_free(plan->d_circ_theta);
        dev_free(plan->d_circ_npar);
        dev_free(plan->d_circ_pool_delta);
        dev_free(plan->d_circ_slot_delta);
        for (void *m : plan->spec_modules) (void)hipModuleUnload((hipModule_t)m);
        delete plan;
    });
}

qsv_status qsv_plan_get_info(const qsv_plan *plan, qsv_plan_info *out)
{
    return guarded([&] {
        if (!plan || !out) fail(QSV_E_ARG, "null argument");
        qsv_plan_info i;
        std::memset(&i, 0, sizeof(i));
        i.n_qubits = plan->n;
        i.n_circuits = plan->n_circuits;
        i.k_local = plan->k;
        i.tile_qubits = plan->t;
        i.reg_qubits = plan->R;
        i.log_threads = plan->LW;
        i.n_gates = (int64_t)plan->gates.size();
        i.n_params = plan->n_params;
        int64_t np = 0;
        for (auto &c : plan->circ) np += (int64_t)c.parts.size();
        i.n_partitions = np;
        i.n_stages = (int64_t)plan->stages.size();
        int64_t P0 = plan->circ.empty() ? 0 : (int64_t)plan->circ[0].parts.size();
        i.ckpt_bytes = plan->n_circuits == 1 && P0 > 1 ? (P0 - 1) * ((int64_t)8 << plan->n) : 0;
        i.flops_per_apply = plan->flops;
        i.bytes_per_apply = plan->bytes;
        i.plan_seconds = plan->plan_seconds;
        i.specialised = plan->specialised ? 1 : 0;
        i.specialise_seconds = plan->specialise_seconds;
        *out = i;
    });
}

qsv_status qsv_plan_specialise(qsv_ctx *ctx, qsv_plan *plan, double *seconds_out)
{
    return guarded([&] {
        if (!plan) fail(QSV_E_ARG, "null plan");
        if (plan->specialised && ctx) {
            if (seconds_out) *seconds_out = plan->specialise_seconds;
            return;
        }
        if (ctx && plan->device != ctx->device) fail(QSV_E_STATE, "plan has no device tables on this context's device");
        if (ctx && plan->async_spec) {  // a background compile is running: wait for it
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            finish_async(*plan, true);
            if (!plan->specialised) fail(QSV_E_DEVICE, plan->specialise_error);
            if (seconds_out) *seconds_out = plan->specialise_seconds;
            return;
        }
        if (plan->n_circuits > 1) {  // batched: one persistent kernel for all circuit structures
            const auto t0 = std::chrono::steady_clock::now();
            std::vector<char> code;
            const std::string err = specialise_batched_compile(*plan, code);
            if (!err.empty()) fail(QSV_E_DEVICE, err);
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (seconds_out) *seconds_out = secs;
            if (!ctx) return;  // compile only
            hip_check(hipSetDevice(ctx->device), "hipSetDevice");
            load_batched(*plan, code);
            plan->specialised = true;
            plan->specialise_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (seconds_out) *seconds_out = plan->specialise_seconds;
            return;
        }
        if (((size_t)8 << plan->t) > (size_t)64 * 1024)
            fail(QSV_E_UNSUPPORTED, "specialised sweeps take tiles of at most 64 KiB of LDS (13 qubits)");
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<SpecChunk> chunks;
        const std::string err = specialise_compile(*plan, chunks, 16);
        if (!err.empty()) fail(QSV_E_DEVICE, err);
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (seconds_out) *seconds_out = secs;
        if (!ctx) return;  // compile only
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        load_spec(*plan, chunks, specialise_reverse(*plan));
        plan->specialised = true;
        plan->specialise_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (seconds_out) *seconds_out = plan->specialise_seconds;
    });
}

qsv_status qsv_plan_specialise_async(qsv_ctx *ctx, qsv_plan *plan)
{
    return guarded([&] {
        if (!ctx || !plan) fail(QSV_E_ARG, "null argument");
        if (plan->specialised || plan->async_spec) return;
        if (plan->n_circuits == 1 && ((size_t)8 << plan->t) > (size_t)64 * 1024)
            fail(QSV_E_UNSUPPORTED, "specialised sweeps take tiles of at most 64 KiB of LDS (13 qubits)");
        if (plan->device != ctx->device) fail(QSV_E_STATE, "plan has no device tables on this context's device");
        auto a = std::make_shared<AsyncSpecialise>();
        a->t0 = std::chrono::steady_clock::now();
        if (plan->n_circuits > 1) {  // batched: the one program of qsv_bspec
            AsyncSpecialise *ap = a.get();
            const Plan *pp = plan;
            ap->chunks.resize(1);
            ap->ready.reset(new std::atomic<bool>[1]);
            ap->ready[0].store(false, std::memory_order_relaxed);
            ap->sized.store(true, std::memory_order_release);
            a->worker = std::thread([ap, pp] {
                try {
                    ap->err = specialise_batched_compile(*pp, ap->chunks[0].code);
                    if (ap->err.empty()) ap->ready[0].store(true, std::memory_order_release);
                } catch (const std::exception &e) {
                    ap->err = std::string("specialise: ") + e.what();
                }
                ap->t1 = std::chrono::steady_clock::now();
            ap->done.store(true, std::memory_order_release);
            });
            plan->async_spec = std::move(a);
            return;
        }
        a->rev = specialise_reverse(*plan);
        AsyncSpecialise *ap = a.get();
        const Plan *pp = plan;
        // small programs (about 48, 16 compiling at a time), the last partitions
        // first: an apply running meanwhile reaches them last
        const int per = std::max(1, ((int)plan->parts.size() + 47) / 48);
        a->worker = std::thread([ap, pp, per] {
            try {
                ap->err = specialise_compile(
                    *pp, ap->chunks, 16, nullptr, per,
                    [ap](size_t c) { ap->ready[c].store(true, std::memory_order_release); },
                    [ap](size_t n) {
                        ap->ready.reset(new std::atomic<bool>[std::max<size_t>(n, 1)]);
                        for (size_t i = 0; i < n; ++i) ap->ready[i].store(false, std::memory_order_relaxed);
                        ap->sized.store(true, std::memory_order_release);
                    });
            } catch (const std::exception &e) {
                ap->err = std::string("specialise: ") + e.what();
            }
            ap->t1 = std::chrono::steady_clock::now();
            ap->done.store(true, std::memory_order_release);
        });
        plan->async_spec = std::move(a);
    });
}

qsv_status qsv_plan_params(const qsv_plan *plan, int32_t circuit, int64_t *offset, int64_t *count)
{
    return guarded([&] {
        if (!plan || !offset || !count) fail(QSV_E_ARG, "null argument");
        if (circuit < 0 || circuit >= plan->n_circuits) fail(QSV_E_ARG, "circuit out of range");
        *offset = plan->circ[circuit].theta_off;
        *count = plan->circ[circuit].n_params;
    });
}

qsv_status qsv_plan_partition(const qsv_plan *plan, int32_t circuit, int32_t level, int64_t p, uint64_t *local_mask,
                              int32_t *gates, int64_t cap, int64_t *n_gates)
{
    return guarded([&] {
        if (!plan || !local_mask || !n_gates) fail(QSV_E_ARG, "null argument");
        if (circuit < 0 || circuit >= plan->n_circuits) fail(QSV_E_ARG, "circuit out of range");
        const CircuitPlan &C = plan->circ[circuit];
        const Part *part = nullptr;
        if (level == -1) {  // distributed partitions: logical local set and logical gate indices
            if (plan->n_global == 0) fail(QSV_E_ARG, "level -1 needs a distributed plan");
            if (p < 0 || p >= (int64_t)plan->dist_parts.size()) fail(QSV_E_ARG, "partition out of range");
            const Part &dp = plan->dist_parts[p];
            *local_mask = dp.S;
            *n_gates = (int64_t)dp.gates.size();
            for (int64_t i = 0; gates && i < std::min<int64_t>(cap, *n_gates); ++i) gates[i] = (int32_t)dp.gates[i];
            return;
        }
        if (level == 0) {
            if (p < 0 || p >= (int64_t)C.parts.size()) fail(QSV_E_ARG, "partition out of range");
            part = &C.parts[p];
        } else if (level == 1) {
            int64_t q = p;
            for (auto &st : C.stages) {
                if (q < (int64_t)st.size()) { part = &st[q]; break; }
                q -= (int64_t)st.size();
            }
            if (!part || p < 0) fail(QSV_E_ARG, "stage out of range");
        } else {
            fail(QSV_E_ARG, "level must be -1, 0 or 1");
        }
        *local_mask = part->S;
        *n_gates = (int64_t)part->gates.size();
        for (int64_t i = 0; gates && i < std::min<int64_t>(cap, *n_gates); ++i) {
            const int64_t g = part->gates[i] - C.g0;
            gates[i] = (int32_t)(plan->n_global ? plan->phys_logical[g] : g);
        }
    });
}

qsv_status qsv_partition_distributed(qsv_ctx *ctx, int32_t n_qubits, const qsv_gate *gates, int64_t n_gates,
                                     int32_t n_global, int32_t k_local, uint32_t flags, const qsv_tile_config *tile,
                                     qsv_plan **out)
{
    return guarded([&] {
        auto t0 = std::chrono::steady_clock::now();
        if (!out) fail(QSV_E_ARG, "out is null");
        if (n_qubits < 2 || n_qubits > (ctx ? MAX_DEVICE_QUBITS : MAX_HOST_QUBITS))
            fail(QSV_E_ARG, ctx ? "n_qubits must be in [2, 35]" : "n_qubits must be in [2, 40] for a host-only plan");
        if (n_gates < 0 || (n_gates > 0 && !gates)) fail(QSV_E_ARG, "bad gate array");
        if (flags & ~(QSV_PLAN_GATE_BY_GATE | QSV_PLAN_GRAD)) fail(QSV_E_ARG, "unknown flag");
        for (int64_t g = 0; g < n_gates; ++g) {
            std::string e = validate_gate(gates[g], n_qubits, 0);
            if (!e.empty()) {
                bool range = e.find("param") != std::string::npos;
                fail(range ? QSV_E_RANGE : QSV_E_ARG, "gate " + std::to_string(g) + ": " + e);
            }
        }
        int R = 4, LW = 8;
        if (tile && (tile->reg_qubits || tile->log_threads)) {
            R = tile->reg_qubits;
            LW = tile->log_threads;
            if (!kernel_shape_supported(R, LW)) fail(QSV_E_ARG, "unsupported tile shape");
        }
        if ((flags & QSV_PLAN_GRAD) && R + LW > 13) fail(QSV_E_UNSUPPORTED, "gradient plans need a tile of at most 13 qubits");
        if (n_global < 1 || n_qubits - n_global < R + LW)
            fail(QSV_E_ARG, "n_global must be >= 1 and leave at least a tile (" + std::to_string(R + LW) +
                                " qubits) local to each rank");
        const int k = k_local == 0 ? R + LW - 3 : k_local;
        if (k >= R + LW) fail(QSV_E_ARG, "k_local must be below the tile size");
        const std::vector<int64_t> off = {0, n_gates};
        qsv_plan *P = make_plan(ctx, n_qubits, gates, off, flags, k, R, LW, n_global);
        P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P;
    });
}

qsv_status qsv_plan_distributed_info(const qsv_plan *plan, int32_t *n_global, int64_t *n_dist_partitions,
                                     int64_t *exchange_swaps, int64_t *remap_swaps)
{
    return guarded([&] {
        if (!plan || !n_global || !n_dist_partitions || !exchange_swaps || !remap_swaps) fail(QSV_E_ARG, "null argument");
        *n_global = plan->n_global;
        *n_dist_partitions = (int64_t)plan->dist_parts.size();
        *exchange_swaps = plan->remap_exchange_swaps;
        *remap_swaps = plan->remap_swaps;
    });
}

qsv_status qsv_apply(qsv_ctx *ctx, const qsv_plan *plan, const double *theta_dev, void *psi_dev, void *ckpt_dev)
{
    return guarded([&] {
        if (!ctx || !plan) fail(QSV_E_ARG, "null ctx or plan");
        if (!psi_dev) fail(QSV_E_ARG, "psi is null");
        if (plan->device != ctx->device || (!plan->d_parts && !plan->parts.empty()))
            fail(QSV_E_STATE, "plan has no device tables on this context's device");
        if (plan->n_params > 0 && !theta_dev) fail(QSV_E_ARG, "theta is null");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        if (plan->n_circuits > 1) {
            finish_async(const_cast<qsv_plan &>(*plan), false);  // a finished background compile
            const int grid = ctx->grid_batched(plan->n_circuits);
            hip_check(launch_batched(*plan, nullptr, 0, nullptr, theta_dev, (float2 *)psi_dev, nullptr, nullptr, nullptr,
                                     nullptr, ctx->ensure_queue(), false, grid, ctx->batch_clock(grid), ctx->stream),
                      "batched launch");
            ctx->last_launches = 0;
            return;
        }
        Plan &mp = const_cast<qsv_plan &>(*plan);
        bool pending = finish_async(mp, false);
        hip_check(launch_materialize(*plan, theta_dev, ctx->stream), "materialize");
        const int np = (int)plan->parts.size();
        if (ctx->timing) {
            while ((int)ctx->events.size() < 2 * np) {
                hipEvent_t e;
                hip_check(hipEventCreate(&e), "hipEventCreate");
                ctx->events.push_back(e);
            }
        }
        float2 *psi = (float2 *)psi_dev;
        float2 *ckpt = (float2 *)ckpt_dev;
        const size_t dim = (size_t)1 << plan->n;
        // a background compile (qsv_plan_specialise_async) may finish during the
        // apply: while it runs, at most two sweeps are queued ahead of the GPU, and
        // each later sweep launches the specialised kernel once it is loaded
        if (pending && !ctx->pace[0]) {
            for (hipEvent_t &e : ctx->pace) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        }
        for (int p = 0; p < np; ++p) {
            if (pending && p >= 2) {
                hip_check(hipEventSynchronize(ctx->pace[p % 2]), "hipEventSynchronize");
                pending = finish_async(mp, false);
            }
            float2 *ck = (ckpt && p < np - 1) ? ckpt + (size_t)p * dim : nullptr;
            if (ctx->timing) hip_check(hipEventRecord(ctx->events[2 * p], ctx->stream), "hipEventRecord");
            hip_check(launch_sweep(*plan, plan->R, plan->LW, p, psi, ck, ctx->stream), "sweep launch");
            if (ctx->timing) hip_check(hipEventRecord(ctx->events[2 * p + 1], ctx->stream), "hipEventRecord");
            if (pending) hip_check(hipEventRecord(ctx->pace[p % 2], ctx->stream), "hipEventRecord");
        }
        ctx->last_launches = ctx->timing ? np : 0;
    });
}

qsv_status qsv_expect(qsv_ctx *ctx, const qsv_pauli_term *H, int32_t n_terms, int32_t n_qubits, int64_t batch,
                      const void *psi_dev, double *out_dev)
{
    return guarded([&] {
        if (!ctx || !psi_dev || !out_dev) fail(QSV_E_ARG, "null argument");
        if (n_qubits < 1 || n_qubits > MAX_DEVICE_QUBITS) fail(QSV_E_ARG, "n_qubits must be in [1, 35]");
        if (batch < 1) fail(QSV_E_ARG, "batch must be >= 1");
        check_terms(H, n_terms, n_qubits);
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        // the same sum as the last call: its tables are still on the device
        std::string key((const char *)H, sizeof(qsv_pauli_term) * (size_t)std::max(0, n_terms));
        key.append((const char *)&n_qubits, sizeof n_qubits);
        if (key != ctx->expect_key) {
            ctx->expect_key.clear();
            HostGroups g = group_terms(H, n_terms, n_qubits, true);
            ctx->expect_dp = nullptr;
            ctx->expect_dg = nullptr;
            ctx->expect_dt = nullptr;
            if (!g.groups.empty())
                upload_groups(ctx, g, ctx->expect_dp, ctx->expect_dg, ctx->expect_dt, &ctx->expect_dev,
                              &ctx->expect_bytes);
            ctx->expect_np = (int)g.passes.size();
            ctx->expect_key = std::move(key);
        }
        size_t need = sizeof(double) * (size_t)expect_blocks(n_qubits) * std::max<size_t>(1, ctx->expect_np) *
                      (size_t)batch;
        double *partials = (double *)ctx->ensure(ctx->scratch, ctx->scratch_bytes, need);
        hip_check(launch_expect(ctx->expect_dp, ctx->expect_np, ctx->expect_dg, ctx->expect_dt, n_qubits, batch,
                                (const float2 *)psi_dev, partials, out_dev, ctx->stream),
                  "expect launch");
    });
}

qsv_status qsv_expect_noalloc(qsv_ctx *ctx, const qsv_pauli_term *H, int32_t n_terms, int32_t n_qubits,
                              int64_t batch, const void *psi_dev, double *out_dev)
{
    return guarded([&] {
        if (!ctx || !psi_dev || !out_dev) fail(QSV_E_ARG, "null argument");
        if (n_qubits < 1 || n_qubits > MAX_DEVICE_QUBITS) fail(QSV_E_ARG, "n_qubits must be in [1, 35]");
        if (batch < 1) fail(QSV_E_ARG, "batch must be >= 1");
        check_terms(H, n_terms, n_qubits);
        if (n_terms > NOALLOC_MAX_TERMS) fail(QSV_E_RANGE, "qsv_expect_noalloc takes at most 4096 Pauli terms");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        char *dev = (char *)noalloc_scratch(ctx->device);
        if (!dev) fail(QSV_E_STATE, "static scratch not set up on this device");
        // the staging buffer is free again once the previous call's copy has run;
        // the grouping of qsv_expect is written straight into it (groups and terms
        // at the offsets of a layout sized for n_terms passes, then the passes)
        hip_check(hipEventSynchronize(ctx->na_staging_ready), "hipEventSynchronize");
        const TermLayout L0 = term_layout((size_t)n_terms, (size_t)n_terms, (size_t)n_terms);
        char *h = (char *)ctx->na_staging;
        int idx[NOALLOC_MAX_TERMS];
        const int n_groups = group_into(H, n_terms, idx, (DevGroup *)(h + L0.groups), (DevTerm *)(h + L0.terms));
        const int n_passes = plan_expect_passes(n_qubits, (DevGroup *)(h + L0.groups), n_groups,
                                                (DevTerm *)(h + L0.terms), (DevPass *)h);
        const size_t partials = sizeof(double) * (size_t)expect_blocks(n_qubits) * (size_t)std::max(1, n_passes) *
                                (size_t)batch;
        if (partials > NOALLOC_SCRATCH_BYTES - NOALLOC_TERMS_BYTES)
            fail(QSV_E_RANGE, "qsv_expect_noalloc: " + std::to_string(partials) + " bytes of partial sums exceed its " +
                                  std::to_string(NOALLOC_SCRATCH_BYTES - NOALLOC_TERMS_BYTES) + "-byte scratch");
        if (n_terms > 0) {
            hip_check(hipMemcpyAsync(dev, h, L0.end, hipMemcpyHostToDevice, ctx->stream), "hipMemcpyAsync");
            hip_check(hipEventRecord(ctx->na_staging_ready, ctx->stream), "hipEventRecord");
        }
        hip_check(launch_expect(n_passes ? (const DevPass *)dev : nullptr, n_passes,
                                n_groups ? (const DevGroup *)(dev + L0.groups) : nullptr,
                                n_groups ? (const DevTerm *)(dev + L0.terms) : nullptr, n_qubits, batch,
                                (const float2 *)psi_dev, (double *)(dev + NOALLOC_TERMS_BYTES), out_dev, ctx->stream),
                  "expect launch");
    });
}

qsv_status qsv_adjoint_grad(qsv_ctx *ctx, const qsv_plan *plan, const qsv_pauli_term *H, int32_t n_terms,
                            const double *theta_dev, const void *psi_final_dev, const void *ckpt_dev,
                            double *energy_dev, double *grad_dev)
{
    return guarded([&] {
        if (!ctx || !plan) fail(QSV_E_ARG, "null ctx or plan");
        if (!energy_dev) fail(QSV_E_ARG, "energy is null");
        if (plan->n_params > 0 && (!theta_dev || !grad_dev)) fail(QSV_E_ARG, "theta or grad is null");
        if (plan->device != ctx->device) fail(QSV_E_STATE, "plan has no device tables on this context's device");
        finish_async(const_cast<qsv_plan &>(*plan), false);  // reverse kernels of a finished background compile
        HostGroups g = group_terms(H, n_terms, plan->n, false);
        DevPass *dp_unused = nullptr;
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        if (plan->n_circuits > 1) {
            const int64_t n_slots = (int64_t)plan->grad_param.size();
            size_t need = sizeof(double) * (size_t)std::max<int64_t>(1, n_slots) * batched_waves();
            double *gpart = (double *)ctx->ensure(ctx->scratch, ctx->scratch_bytes, need);
            DevGroup *dg = nullptr;
            DevTerm *dt = nullptr;
            if (!g.groups.empty()) upload_groups(ctx, g, dp_unused, dg, dt);
            const int grid = ctx->grid_batched(plan->n_circuits);
            const float2 *psi_in = (const float2 *)psi_final_dev;
            if (!psi_in && plan->spec_batch_fn) {
                // the specialised forward into a scratch batch of states, then the
                // adjoint walk (table-driven) from them
                const size_t bytes = ((size_t)plan->n_circuits << plan->n) * sizeof(float2);
                float2 *states = (float2 *)ctx->ensure(ctx->lam, ctx->lam_bytes, bytes);
                hip_check(launch_batched(*plan, nullptr, 0, nullptr, theta_dev, states, nullptr, nullptr, nullptr,
                                         nullptr, ctx->ensure_queue(), false, grid, nullptr, ctx->stream),
                          "batched launch");
                psi_in = states;
            }
            hip_check(launch_batched(*plan, dg, (int)g.groups.size(), dt, theta_dev, nullptr, psi_in, energy_dev,
                                     grad_dev, gpart, ctx->ensure_queue(), true, grid, ctx->batch_clock(grid),
                                     ctx->stream),
                      "batched launch");
            return;
        }
        if (!(plan->flags & QSV_PLAN_GRAD)) fail(QSV_E_STATE, "plan was built without QSV_PLAN_GRAD");
        if (!psi_final_dev) fail(QSV_E_ARG, "psi_final is null");
        const int np = (int)plan->parts.size();
        if (np > 1 && !ckpt_dev) fail(QSV_E_STATE, "checkpoints missing");
        const int n = plan->n;
        const size_t dim = (size_t)1 << n;
        // scratch: lambda state + reduction partials + gradient partials
        float2 *lam = (float2 *)ctx->ensure(ctx->lam, ctx->lam_bytes, dim * sizeof(float2));
        const int n_blocks = 4096;  // cap on the blocks of lambda = H psi
        const int t = plan->t;
        const int64_t n_tiles = (int64_t)1 << (n - t);
        const int64_t waves = std::max(1, (1 << plan->LW) / 64);
        const int64_t n_slots = (int64_t)plan->grad_param.size();
        size_t red = sizeof(double) * (size_t)apply_h_blocks(n, n_blocks);
        size_t gp = sizeof(double) * (size_t)std::max<int64_t>(1, n_slots) * n_tiles * waves;
        size_t sl = sizeof(double) * (size_t)std::max<int64_t>(1, n_slots);
        const size_t gp_off = (red + 255) & ~size_t(255), sl_off = (gp_off + gp + 255) & ~size_t(255);
        char *scr = (char *)ctx->ensure(ctx->scratch, ctx->scratch_bytes, sl_off + sl);
        double *partials = (double *)scr;
        double *gpart = (double *)(scr + gp_off);
        double *slot_sum = (double *)(scr + sl_off);
        DevGroup *dg = nullptr;
        DevTerm *dt = nullptr;
        if (!g.groups.empty()) upload_groups(ctx, g, dp_unused, dg, dt);
        hip_check(launch_materialize(*plan, theta_dev, ctx->stream), "materialize");
        hip_check(launch_apply_h(dg, (int)g.groups.size(), dt, n, (const float2 *)psi_final_dev, lam, partials,
                                 n_blocks, energy_dev, ctx->stream),
                  "apply_h launch");
        for (int p = np - 1; p >= 0; --p) {
            const float2 *src = p == np - 1 ? (const float2 *)psi_final_dev : (const float2 *)ckpt_dev + (size_t)p * dim;
            hip_check(launch_reverse(*plan, plan->R, plan->LW, p, src, lam, gpart, n_tiles * waves, ctx->stream),
                      "reverse launch");
        }
        if (plan->n_params > 0)
            hip_check(launch_grad_reduce(*plan, gpart, n_slots, n_tiles * waves, slot_sum, grad_dev, ctx->stream),
                      "grad reduce");
    });
}

}  // extern "C"
