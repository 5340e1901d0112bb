// C ABI of the sampler: state management, the sweep schedule, graphs and
// the device-resident draw ring.  See include/hsp.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "../../include/hsp.h"
#include "../../include/hsp_diag.h"
#include "hsp_internal.hpp"
#include "tune.hpp"

using namespace hsp;

namespace {
thread_local std::string g_create_error;

// Launch timing with HIP events on one stream: a pair of events around each
// timed launch, from a pool of kPairs pairs; when the pool is full its
// durations are folded into a running sum (waiting for the last of them), so
// a long timed run holds a bounded number of events.
struct EventTimer {
    static constexpr size_t kPairs = 256;
    std::vector<hipEvent_t> pool;  // 2 kPairs events, created on first use
    hipEvent_t first = nullptr;    // recorded before the first timed launch
    size_t used = 0;               // pairs recorded since the last fold
    size_t last = 0;               // pool index of the latest end event
    double sum_ms = 0.0;           // durations of folded pairs
    int64_t n = 0;                 // timed launches

    hipError_t fold() {
        if (!used) return hipSuccess;
        hipError_t e = hipEventSynchronize(pool[2 * used - 1]);
        for (size_t i = 0; !e && i < used; ++i) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, pool[2 * i], pool[2 * i + 1]);
            sum_ms += ms;
        }
        used = 0;
        return e;
    }
    hipError_t begin(hipStream_t st) {
        if (pool.empty()) {
            pool.assign(2 * kPairs, nullptr);
            for (auto& e : pool)
                if (hipError_t r = hipEventCreate(&e)) return r;
            if (hipError_t r = hipEventCreate(&first)) return r;
        }
        if (used == kPairs)
            if (hipError_t r = fold()) return r;
        if (n == 0)
            if (hipError_t r = hipEventRecord(first, st)) return r;
        return hipEventRecord(pool[2 * used], st);
    }
    hipError_t end(hipStream_t st) {
        last = 2 * used + 1;
        ++used;
        ++n;
        return hipEventRecord(pool[last], st);
    }
    // Mean duration per launch and (first start to last end) / launches.
    hipError_t result(double* mean_ms, double* span_ms, int64_t* count) {
        *mean_ms = *span_ms = 0.0;
        *count = n;
        if (!n) return hipSuccess;
        if (hipError_t e = fold()) return e;
        float ms = 0.0f;
        if (hipError_t e = hipEventElapsedTime(&ms, first, pool[last])) return e;
        *mean_ms = sum_ms / n;
        *span_ms = ms / n;
        return hipSuccess;
    }
    void reset() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        if (first) (void)hipEventDestroy(first);
        pool.clear();
        first = nullptr;
        used = last = 0;
        sum_ms = 0.0;
        n = 0;
    }
};
}  // namespace

struct hsp_state {
    int device = 0;
    int num_cus = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hsp_options opt{};
    XLayout x{};
    void* Xbuf = nullptr;
    int32_t* xexp = nullptr;        // p: column j of Xbuf is stored times 2^-xexp[j]
    double* xscale = nullptr;       // p: 2^xexp[j]
    std::vector<double> xscale_h;   // host copy of xscale
    uint8_t* y = nullptr;
    Ctrl* ctrl = nullptr;
    double *beta = nullptr, *lam = nullptr, *nu = nullptr, *tau = nullptr, *xi = nullptr;
    double *b = nullptr, *G = nullptr, *Gp = nullptr, *A = nullptr, *Linv = nullptr;
    double *vec = nullptr, *partial = nullptr, *bsum = nullptr;
    uint32_t* zgrp_count = nullptr;
    uint32_t *tasks = nullptr, *task_off = nullptr, *ver = nullptr;  // tile path schedule
    float* beta32 = nullptr;
    float* zdbg = nullptr;
    int32_t* adbg = nullptr;
    double *ring_beta = nullptr, *ring_tau = nullptr, *ring_lam = nullptr;
    SweepPlan plan{};
    uint64_t timeout_ticks = 0;
    uint64_t sweeps_done = 0;  // host mirror of ctrl->sweep
    uint64_t draw_base = 0;    // host mirror of ctrl->draw_base
    std::string err;
    bool poisoned = false;
    hipGraphExec_t graph = nullptr;  // one whole sweep (one kernel), recording
    uint64_t* trace = nullptr;        // p-side phase timestamps (diagnostics)
    SweepArgs* dargs = nullptr;       // [0]: a whole sweep, [1]: the last hsp_step
    const SweepArgs** dtab = nullptr;  // device table {dargs, dargs + 1} for the launches
    const hsp_state* owner = nullptr;  // batch chain: X, y, G, Gp belong to this state
    bool in_batch = false;             // owned by an hsp_batch (not destroyed alone)
    bool timing = false;
    EventTimer timer;  // timed sweeps
    std::string plan_note;  // how the launch plan was chosen (autotuner)
    // X streamed from pinned host memory in row chunks (x_stream)
    bool streamed = false;
    void* Xhost = nullptr;              // N x ld library layout, pinned
    void* stage[2] = {nullptr, nullptr};  // device chunk buffers
    uint32_t chunk_rows = 0, nchunks = 0;
    hipStream_t copy_stream = nullptr;  // the chunks' host-to-device copies
    hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    bool freed_used[2] = {false, false};
    SweepArgs* sdargs = nullptr;        // nchunks z-pass launches + the p-side launch (device)
    const SweepArgs** sdtab = nullptr;
    std::vector<SweepArgs> sd_host;     // host copies of the same
    uint32_t sd_mode = 0;               // the mode they were built for (0: none yet)
    uint32_t* row_id = nullptr;         // original index of each stored row once reordered (device)
};

namespace {

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) return fail_hip(s, #expr, e_);                          \
    } while (0)

hsp_status fail(hsp_state* s, hsp_status code, const std::string& msg) {
    if (s) {
        s->err = msg;
        if (code == HSP_EHIP || code == HSP_ENOTPD || code == HSP_ERANGE) s->poisoned = true;
    } else {
        g_create_error = msg;
    }
    return code;
}

hsp_status fail_hip(hsp_state* s, const char* what, hipError_t e) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(s, HSP_ENOMEM, m);
    return fail(s, HSP_EHIP, m);
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

SweepArgs sweep_args(hsp_state* s, uint32_t mode) {
    SweepArgs a{};
    a.x = s->x;
    a.y = dev_ptr(s->y);
    a.beta32 = dev_ptr(s->beta32);
    a.xscale = dev_ptr(static_cast<const double*>(s->xscale));
    a.partial = dev_ptr(s->partial);
    a.bsum = dev_ptr(s->bsum);
    a.zgrp_count = dev_ptr(s->zgrp_count);
    a.zdbg = dev_ptr(s->opt.debug_store_z ? s->zdbg : nullptr);
    a.adbg = dev_ptr(s->opt.debug_store_z ? s->adbg : nullptr);
    a.beta = dev_ptr(s->beta);
    a.lam_m2 = dev_ptr(s->lam);
    a.nu_m1 = dev_ptr(s->nu);
    a.tau_m2 = dev_ptr(s->tau);
    a.xi_m1 = dev_ptr(s->xi);
    a.b = dev_ptr(s->b);
    a.G = dev_ptr(s->G);
    a.Gp = dev_ptr(s->Gp);
    a.A = dev_ptr(s->A);
    a.Linv = dev_ptr(s->Linv);
    a.tasks = dev_ptr(s->tasks);
    a.task_off = dev_ptr(s->task_off);
    a.ver = dev_ptr(s->ver);
    a.row_id = dev_ptr(static_cast<const uint32_t*>(s->row_id));
    a.vec = dev_ptr(s->vec);
    a.ring_beta = dev_ptr(s->ring_beta);
    a.ring_tau = dev_ptr(s->ring_tau);
    a.ring_lam = dev_ptr(s->ring_lam);
    a.thin = (uint32_t)s->opt.thin;
    a.capacity = (uint32_t)s->opt.max_draws;
    a.ctrl = dev_ptr(s->ctrl);
    a.seed = s->opt.seed;
    a.chain = s->opt.chain_id;
    a.mode = mode;
    a.timeout_ticks = s->timeout_ticks;
    a.trace = dev_ptr(s->trace);
    a.gp = a.gz = a.zgroups = a.block0 = a.idle = 0;
    const uint32_t nt = (s->x.p + kTile - 1) / kTile;
    a.subst = s->x.p > (uint32_t)kSmallP && !with_inverse(nt) ? 1u : 0u;
    return a;
}

// Upload the launch description of `mode` into device slot `slot`.
hipError_t put_args(hsp_state* s, uint32_t mode, int slot, SweepArgs* out) {
    *out = sweep_args(s, mode);
    sweep_finish_args(out, s->plan);
    return hipMemcpy(s->dargs + slot, out, sizeof(SweepArgs), hipMemcpyHostToDevice);
}

constexpr uint32_t kModeSweep =
    kModeZ | kModeLambda | kModeTau | kModeBeta | kModeNuXi | kModeRecord | kModeAdvance;

hipError_t enqueue_sweep(hsp_state* s, hipStream_t st) {
    SweepArgs h = sweep_args(s, kModeSweep);
    sweep_finish_args(&h, s->plan);
    return sweep_launch(h, s->dtab, s->plan, st);
}

hipError_t capture(hsp_state* s, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e) return e;
    hipError_t e2 = enqueue_sweep(s, s->stream);
    e = hipStreamEndCapture(s->stream, &g);
    if (e2) {
        if (g) (void)hipGraphDestroy(g);
        return e2;
    }
    if (e) return e;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

hsp_status check_device_flags(hsp_state* s) {
    Ctrl c;
    HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (c.err & kErrNotPD) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "X^T X + tau^-2 Lambda^-2 is not positive definite (pivot %d) at sweep %u",
                      c.chol_info, c.sweep + 1);
        return fail(s, HSP_ENOTPD, buf);
    }
    if (c.err & kErrTnCap)
        return fail(s, HSP_ERANGE, "a truncated-normal row reached the proposal cap (non-finite X beta)");
    if (c.err & kErrNonFinite) return fail(s, HSP_ERANGE, "a draw of beta, lambda or tau was not finite");
    if (c.err & kErrTimeout)
        return fail(s, HSP_EHIP, "a bounded wait inside the sweep kernel timed out");
    return HSP_OK;
}

hsp_status sync_state(hsp_state* s) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    return check_device_flags(s);
}

void free_state(hsp_state* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->timer.reset();
    if (s->owner) {  // borrowed from the dataset's first chain
        s->Xbuf = nullptr;
        s->xexp = nullptr;
        s->xscale = nullptr;
        s->y = nullptr;
        s->G = nullptr;
        s->Gp = nullptr;
    }
    void* bufs[] = {s->Xbuf, s->xexp, s->xscale, s->y, s->ctrl, s->beta, s->lam, s->nu, s->tau, s->xi, s->b, s->G, s->Gp,
                    s->A, s->Linv, s->vec, s->partial, s->beta32, s->zdbg, s->adbg,
                    s->ring_beta, s->ring_tau, s->ring_lam, s->trace, s->bsum,
                    s->zgrp_count, s->dargs, s->dtab, s->tasks, s->task_off, s->ver, s->row_id};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (s->streamed) {
        // s->Xbuf is null for a streamed state: X lives in Xhost and the stages
        if (s->Xhost) (void)hipHostFree(s->Xhost);
        for (int i = 0; i < 2; ++i) {
            if (s->stage[i]) (void)hipFree(s->stage[i]);
            if (s->copied[i]) (void)hipEventDestroy(s->copied[i]);
            if (s->freed[i]) (void)hipEventDestroy(s->freed[i]);
        }
        if (s->sdargs) (void)hipFree(s->sdargs);
        if (s->sdtab) (void)hipFree(s->sdtab);
        if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    }
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

hsp_status upload_state(hsp_state* s, const double* beta, const double* lam, const double* nu,
                        double tau, double xi) {
    const uint32_t p = s->x.p;
    std::vector<float> b32(s->x.ld, 0.0f);
    for (uint32_t j = 0; j < p; ++j) b32[j] = (float)(beta[j] * s->xscale_h[j]);
    HIP_TRY(hipMemcpy(s->beta, beta, p * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->beta32, b32.data(), s->x.ld * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->lam, lam, p * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->nu, nu, p * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->tau, &tau, sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->xi, &xi, sizeof(double), hipMemcpyHostToDevice));
    return HSP_OK;
}

hsp_status set_counters(hsp_state* s, uint64_t sweep) {
    Ctrl c;
    HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    c.sweep = (uint32_t)sweep;
    c.draw_base = (uint32_t)sweep;
    c.bar_count = c.bar_epoch = 0;
    c.z_count = c.z_epoch = 0;
    HIP_TRY(hipMemcpy(s->ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice));
    s->sweeps_done = sweep;
    s->draw_base = sweep;
    return HSP_OK;
}

hsp_status chain_impl(hsp_state* s);

// The factorisation's task lists for the plan's group size (tile path).
hsp_status upload_schedule(hsp_state* s) {
    const uint32_t nt = (s->x.p + kTile - 1) / kTile;
    std::vector<uint32_t> tasks, off;
    chol_schedule(nt, s->plan.gp, &tasks, &off, with_inverse(nt));
    if (s->tasks) (void)hipFree(s->tasks);
    if (s->task_off) (void)hipFree(s->task_off);
    s->tasks = s->task_off = nullptr;
    HIP_TRY(dalloc(&s->tasks, tasks.size()));
    HIP_TRY(dalloc(&s->task_off, off.size()));
    HIP_TRY(hipMemcpy(s->tasks, tasks.data(), tasks.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->task_off, off.data(), off.size() * 4, hipMemcpyHostToDevice));
    return HSP_OK;
}

// Switch the state to another launch plan (the next sweep uses it).
hsp_status apply_plan(hsp_state* s, const SweepPlan& plan) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    const bool regroup = plan.gp != s->plan.gp;
    s->plan = plan;
    if (regroup && s->x.p > (uint32_t)kSmallP) {
        hsp_status st = upload_schedule(s);
        if (st) return st;
    }
    SweepArgs h;
    HIP_TRY(put_args(s, kModeSweep, 0, &h));
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    return HSP_OK;
}

std::string device_tag(int device, int num_cus) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == '\t' || c == ' ' || c == '\n') c = '_';
    return arch + " cus=" + std::to_string(num_cus);
}

// Cache key of a single chain's plan: the device, the shape and the plan format.
std::string sweep_tune_key(const hsp_state* s) {
    return "sweep-v1 " + device_tag(s->device, s->num_cus) + " xt=" + std::to_string(s->x.xtype) +
           " N=" + std::to_string(s->x.N) + " p=" + std::to_string(s->x.p);
}

const char* tune_cache_path() {
    const char* p = std::getenv("HSP_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// Mean milliseconds of `timed` launches of the sweep kernel after `warm`
// untimed ones, on the state's stream.
hsp_status time_sweeps(hsp_state* s, int warm, int timed, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    for (int i = 0; !e && i < warm; ++i) e = enqueue_sweep(s, s->stream);
    if (!e) e = hipEventRecord(e0, s->stream);
    for (int i = 0; !e && i < timed; ++i) e = enqueue_sweep(s, s->stream);
    if (!e) e = hipEventRecord(e1, s->stream);
    if (!e) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (!e) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    HIP_TRY(e);
    *ms = (double)t / timed;
    return check_device_flags(s);
}

// The Markov state and control block of a chain, kept on the host while the
// autotuner runs sweeps, then put back.
struct SavedChain {
    std::vector<double> beta, lam, nu;
    double tau = 0.0, xi = 0.0;
    Ctrl ctrl{};
};

hsp_status save_chain(hsp_state* s, SavedChain* c) {
    const size_t p = s->x.p;
    c->beta.resize(p);
    c->lam.resize(p);
    c->nu.resize(p);
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(c->beta.data(), s->beta, p * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(c->lam.data(), s->lam, p * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(c->nu.data(), s->nu, p * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&c->tau, s->tau, 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&c->xi, s->xi, 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&c->ctrl, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    return HSP_OK;
}

hsp_status restore_chain(hsp_state* s, const SavedChain& c) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    hsp_status st = upload_state(s, c.beta.data(), c.lam.data(), c.nu.data(), c.tau, c.xi);
    if (st) return st;
    HIP_TRY(hipMemcpy(s->ctrl, &c.ctrl, sizeof(Ctrl), hipMemcpyHostToDevice));
    return HSP_OK;
}

// A plan read back from the cache, if it is one this state can run.
bool plan_from_text(hsp_state* s, const std::string& v, SweepPlan* out) {
    long gp = 0, pct = 0, unit = 0;
    if (!tune_parse(v, "gp", &gp) || !tune_parse(v, "pct", &pct) || !tune_parse(v, "unit", &unit)) return false;
    if (gp < 1 || pct < 0 || pct > 100 || unit < 1 || unit > (long)kZUnitMax) return false;
    SweepPlan pl;
    if (sweep_plan(s->x, s->num_cus, &pl, (uint32_t)gp) != hipSuccess || pl.gp != (uint32_t)gp) return false;
    pl.static_pct = (uint32_t)pct;
    pl.unit = (uint32_t)unit;
    *out = pl;
    return true;
}

std::string plan_text(const SweepPlan& pl) {
    return "gp=" + std::to_string(pl.gp) + " pct=" + std::to_string(pl.static_pct) + " unit=" +
           std::to_string(pl.unit);
}

// The autotuner for one chain: the p-side group size and how the z pass deals
// out its tiles, by timing a few sweeps of every candidate (or from the cache).
hsp_status tune_impl(hsp_state* s) {
    const std::string key = sweep_tune_key(s);
    const char* path = tune_cache_path();
    std::string cached;
    SweepPlan pl;
    if (path && tune_cache_get(path, key, &cached) && plan_from_text(s, cached, &pl)) {
        s->plan_note = plan_text(pl) + " (cache)";
        return apply_plan(s, pl);
    }
    SavedChain saved;
    hsp_status st = save_chain(s, &saved);
    if (st) return st;
    const uint32_t gmax = max_group(s->x, s->plan.capacity);
    // beyond p = 4096 the factorisation sets the pace: only the group size is
    // tried (each size builds a task schedule of ~p^3 / 10^5 tasks)
    const bool large = s->x.p > kLargeP;
    std::vector<uint32_t> gps{gmax};
    if (s->x.p > (uint32_t)kSmallP)
        for (uint32_t pct : large ? std::vector<uint32_t>{67u} : std::vector<uint32_t>{75u, 50u, 33u}) {
            const uint32_t g = std::max<uint32_t>(1, (gmax * pct + 50) / 100);
            if (std::find(gps.begin(), gps.end(), g) == gps.end()) gps.push_back(g);
        }
    // where the factorisation was judged to outweigh the pass, the smaller
    // group that would otherwise be chosen is tried as well
    if (!large && s->x.p > (uint32_t)kSmallP) {
        const uint32_t q = std::max<uint32_t>(1, std::min<uint32_t>(kMaxGroup, (uint32_t)s->plan.capacity / 4));
        if (q < gmax && std::find(gps.begin(), gps.end(), q) == gps.end()) gps.push_back(q);
    }
    const std::vector<uint32_t> pcts = large ? std::vector<uint32_t>{kZStaticPctDefault}
                                             : std::vector<uint32_t>{0u, 40u, 75u};
    const std::vector<uint32_t> units = large ? std::vector<uint32_t>{kZUnitDefault}
                                              : std::vector<uint32_t>{4u, 8u, 16u};
    // shorter runs for big designs: every candidate sweeps all of X
    const double bytes = (double)s->x.N * s->x.ld * (s->x.xtype == 0 ? 4 : 2);
    const int timed = bytes > 1e10 ? 3 : bytes > 1e9 ? 4 : 8;
    SweepPlan best = s->plan;
    double best_ms = 1e300;
    for (uint32_t gp : gps)
        for (uint32_t pct : pcts)
            for (uint32_t unit : units) {
                SweepPlan c;
                HIP_TRY(sweep_plan(s->x, s->num_cus, &c, gp));
                c.static_pct = pct;
                c.unit = unit;
                st = apply_plan(s, c);
                double ms = 0.0;
                if (!st) st = time_sweeps(s, 2, timed, &ms);
                if (st) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    st = apply_plan(s, best);
    if (!st) st = restore_chain(s, saved);
    if (st) return st;
    char buf[64];
    std::snprintf(buf, sizeof buf, " ms=%.4f", best_ms);
    s->plan_note = plan_text(best) + buf + " (measured)";
    if (path) (void)tune_cache_put(path, key, plan_text(best) + buf);
    return HSP_OK;
}

// Device, stream and wait bound of a new state.
hsp_status setup_impl(hsp_state* s) {
    HIP_TRY(hipGetDevice(&s->device));
    HIP_TRY(hipDeviceGetAttribute(&s->num_cus, hipDeviceAttributeMultiprocessorCount, s->device));
    {
        // every wait inside the sweep kernel gives up after 2 seconds
        int khz = 0;
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device));
        if (khz <= 0) khz = 100000;
        s->timeout_ticks = (uint64_t)khz * 1000ull * 2ull;
    }
    if (s->opt.hip_stream) {
        s->stream = static_cast<hipStream_t>(s->opt.hip_stream);
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    return HSP_OK;
}

hsp_status create_impl(hsp_state* s, const float* X, const uint8_t* y, int64_t N, int64_t p) {
    hsp_status st0 = setup_impl(s);
    if (st0) return st0;
    const int xt = s->opt.x_type;
    const uint32_t align = xt == HSP_X_F32 ? 4 : 8;
    const uint32_t ld = (uint32_t)((p + align - 1) / align * align);
    const size_t esz = xt == HSP_X_F32 ? 4 : 2;
    HIP_TRY(hipMalloc(&s->Xbuf, (size_t)N * ld * esz));
    s->x.X = dev_ptr(static_cast<const void*>(s->Xbuf));
    s->x.xtype = xt;
    s->x.N = (uint32_t)N;
    s->x.p = (uint32_t)p;
    s->x.ld = ld;
    HIP_TRY(dalloc(&s->y, (size_t)N));
    HIP_TRY(dalloc(&s->ctrl, 1));
    HIP_TRY(hipMemsetAsync(s->ctrl, 0, sizeof(Ctrl), s->stream));
    const hipMemcpyKind kind = s->opt.x_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;

    // X into the library layout, column j scaled by 2^-e_j so that its
    // largest magnitude lies in (1/2, 1]: the column maxima come first, from
    // the float32 source on the device (the caller's X, a staging copy of a
    // host X, or the library buffer itself when the layouts coincide).
    HIP_TRY(dalloc(&s->xexp, (size_t)p));
    HIP_TRY(dalloc(&s->xscale, (size_t)p));
    {
        const bool inplace = xt == HSP_X_F32 && ld == (uint32_t)p;
        float* stage = nullptr;
        const float* src = X;
        if (inplace) {
            HIP_TRY(hipMemcpyAsync(s->Xbuf, X, (size_t)N * p * 4, kind, s->stream));
            src = static_cast<const float*>(s->Xbuf);
        } else if (s->opt.x_on_host) {
            HIP_TRY(dalloc(&stage, (size_t)N * p));
            src = stage;
        }
        uint32_t* cm = nullptr;
        hipError_t e = dalloc(&cm, (size_t)p);
        if (!e && stage) e = hipMemcpyAsync(stage, X, (size_t)N * p * 4, kind, s->stream);
        if (!e) e = hipMemsetAsync(cm, 0, (size_t)p * 4, s->stream);
        if (!e) e = colmax_launch(src, (uint32_t)N, (uint32_t)p, cm, s->stream);
        std::vector<uint32_t> bits(p);
        if (!e) e = hipMemcpyAsync(bits.data(), cm, (size_t)p * 4, hipMemcpyDeviceToHost, s->stream);
        if (!e) e = hipStreamSynchronize(s->stream);
        std::vector<int32_t> ex(p, 0);
        s->xscale_h.assign(p, 1.0);
        for (int64_t j = 0; !e && j < p; ++j) {
            // a zero or non-finite column keeps scale 1 (non-finite X is rejected below)
            if (bits[j] == 0 || bits[j] >= 0x7F800000u) continue;
            float m;
            std::memcpy(&m, &bits[j], 4);
            int k = 0;
            const float f = std::frexp(m, &k);  // m = f 2^k, f in [1/2, 1)
            ex[j] = f == 0.5f ? k - 1 : k;
            s->xscale_h[j] = std::ldexp(1.0, ex[j]);
        }
        if (!e) e = hipMemcpyAsync(s->xexp, ex.data(), (size_t)p * 4, hipMemcpyHostToDevice, s->stream);
        if (!e) e = hipMemcpyAsync(s->xscale, s->xscale_h.data(), (size_t)p * 8, hipMemcpyHostToDevice,
                                   s->stream);
        if (!e) e = pack_x_launch(src, s->x, s->xexp, s->stream);
        if (!e) e = hipStreamSynchronize(s->stream);
        if (cm) (void)hipFree(cm);
        if (stage) (void)hipFree(stage);
        HIP_TRY(e);
    }
    HIP_TRY(hipMemcpyAsync(s->y, y, (size_t)N, kind, s->stream));
    HIP_TRY(validate_launch(s->x, s->y, s->ctrl, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    {
        Ctrl c;
        HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (c.err & kErrInput)
            return fail(nullptr, HSP_EINVAL,
                        "y must hold only 0/1 and X must be finite (also after bfloat16 rounding)");
    }

    // G = X^T X (and Gp for the tiled path), shared by every chain of this data
    HIP_TRY(dalloc(&s->G, (size_t)p * p));
    const size_t P = ((size_t)p + kTile - 1) / kTile * kTile;
    if (p > kSmallP) HIP_TRY(dalloc(&s->Gp, P * P));
    {
        double* work = nullptr;
        HIP_TRY(dalloc(&work, gram_work_doubles(s->x, s->num_cus)));
        hipError_t e = gram_launch(s->x, s->xexp, s->G, work, s->num_cus, s->stream);
        if (!e && s->Gp) e = pad_gram_launch(s->G, (uint32_t)p, (uint32_t)P, s->Gp, s->stream);
        if (!e) e = hipStreamSynchronize(s->stream);
        (void)hipFree(work);
        HIP_TRY(e);
    }
    return chain_impl(s);
}

// X kept in pinned host memory and streamed through the GPU (x_stream).
// Creation makes two passes over X in chunks of whole Gram row splits, with
// the same kernels as the resident path: the column maxima, then each chunk
// scaled (and rounded to bfloat16) into the library layout, validated, its
// Gram partial tiles formed, and copied out to the pinned buffer.  G is then
// summed over the splits in order, as for a resident X.
hsp_status create_stream_impl(hsp_state* s, const float* X, const uint8_t* y, int64_t N, int64_t p) {
    hsp_status st0 = setup_impl(s);
    if (st0) return st0;
    s->streamed = true;
    const int xt = s->opt.x_type;
    const uint32_t align = xt == HSP_X_F32 ? 4 : 8;
    const uint32_t ld = (uint32_t)((p + align - 1) / align * align);
    const size_t esz = xt == HSP_X_F32 ? 4 : 2;
    const size_t row_bytes = (size_t)ld * esz;
    uint64_t budget = s->opt.stream_rows > 0 ? (uint64_t)s->opt.stream_rows
                                             : std::max<uint64_t>(64, ((uint64_t)256 << 20) / row_bytes);
    budget = std::max<uint64_t>(64, budget / 64 * 64);
    XLayout full{};
    full.xtype = xt;
    full.N = (uint32_t)N;
    full.p = (uint32_t)p;
    full.ld = ld;
    const GramGeometry gg = gram_geometry(full, s->num_cus, budget);
    const uint64_t per = std::max<uint64_t>(1, budget / gg.rows_per_split);
    s->chunk_rows = (uint32_t)std::min<uint64_t>((uint64_t)gg.rows_per_split * per,
                                                 ((uint64_t)N + 63) / 64 * 64);
    s->nchunks = (uint32_t)(((uint64_t)N + s->chunk_rows - 1) / s->chunk_rows);
    HIP_TRY(hipHostMalloc(&s->Xhost, (size_t)N * row_bytes, hipHostMallocDefault));
    for (int i = 0; i < 2; ++i) HIP_TRY(dalloc(reinterpret_cast<char**>(&s->stage[i]), (size_t)s->chunk_rows * row_bytes));
    s->x = full;
    s->x.X = dev_ptr(static_cast<const void*>(s->stage[0]));
    HIP_TRY(dalloc(&s->y, (size_t)N));
    HIP_TRY(dalloc(&s->ctrl, 1));
    HIP_TRY(hipMemsetAsync(s->ctrl, 0, sizeof(Ctrl), s->stream));
    const hipMemcpyKind kind = s->opt.x_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(s->y, y, (size_t)N, kind, s->stream));
    HIP_TRY(dalloc(&s->xexp, (size_t)p));
    HIP_TRY(dalloc(&s->xscale, (size_t)p));
    // float32 source of a chunk: the caller's device X in place, or a staged host chunk
    float* raw = nullptr;
    if (s->opt.x_on_host) HIP_TRY(dalloc(&raw, (size_t)s->chunk_rows * p));
    uint32_t* cm = nullptr;
    double* work = nullptr;
    hipError_t e = dalloc(&cm, (size_t)p);
    auto source = [&](uint32_t c, uint32_t* rows) -> const float* {
        const size_t r0 = (size_t)c * s->chunk_rows;
        *rows = (uint32_t)std::min<size_t>(s->chunk_rows, (size_t)N - r0);
        if (!raw) return X + r0 * p;
        if (!e) e = hipMemcpyAsync(raw, X + r0 * p, (size_t)*rows * p * 4, kind, s->stream);
        return raw;
    };
    if (!e) e = hipMemsetAsync(cm, 0, (size_t)p * 4, s->stream);
    for (uint32_t c = 0; !e && c < s->nchunks; ++c) {
        uint32_t rows = 0;
        const float* src = source(c, &rows);
        if (!e) e = colmax_launch(src, rows, (uint32_t)p, cm, s->stream);
    }
    std::vector<uint32_t> bits(p);
    if (!e) e = hipMemcpyAsync(bits.data(), cm, (size_t)p * 4, hipMemcpyDeviceToHost, s->stream);
    if (!e) e = hipStreamSynchronize(s->stream);
    std::vector<int32_t> ex(p, 0);
    s->xscale_h.assign(p, 1.0);
    for (int64_t j = 0; !e && j < p; ++j) {
        if (bits[j] == 0 || bits[j] >= 0x7F800000u) continue;
        float m;
        std::memcpy(&m, &bits[j], 4);
        int k = 0;
        const float f = std::frexp(m, &k);
        ex[j] = f == 0.5f ? k - 1 : k;
        s->xscale_h[j] = std::ldexp(1.0, ex[j]);
    }
    if (!e) e = hipMemcpyAsync(s->xexp, ex.data(), (size_t)p * 4, hipMemcpyHostToDevice, s->stream);
    if (!e) e = hipMemcpyAsync(s->xscale, s->xscale_h.data(), (size_t)p * 8, hipMemcpyHostToDevice, s->stream);
    if (!e) e = dalloc(&work, (size_t)gg.nsplit * gg.npairs * kTile * kTile);
    for (uint32_t c = 0; !e && c < s->nchunks; ++c) {
        uint32_t rows = 0;
        const float* src = source(c, &rows);
        XLayout cl = full;
        cl.X = dev_ptr(static_cast<const void*>(s->stage[0]));
        cl.N = rows;
        const size_t r0 = (size_t)c * s->chunk_rows;
        if (!e) e = pack_x_launch(src, cl, s->xexp, s->stream);
        if (!e) e = validate_launch(cl, s->y + r0, s->ctrl, s->stream);
        if (!e) e = gram_chunk_launch(cl, gg, (uint32_t)(r0 / gg.rows_per_split), work, s->stream);
        if (!e) e = hipMemcpyAsync(static_cast<char*>(s->Xhost) + r0 * row_bytes, s->stage[0], rows * row_bytes,
                                   hipMemcpyDeviceToHost, s->stream);
        if (!e) e = hipStreamSynchronize(s->stream);  // the stage and raw buffers are reused
    }
    if (!e) e = dalloc(&s->G, (size_t)p * p);
    if (!e) e = gram_reduce_launch(work, gg, (uint32_t)p, s->xexp, s->G, s->stream);
    const size_t P = ((size_t)p + kTile - 1) / kTile * kTile;
    if (!e && p > kSmallP) e = dalloc(&s->Gp, P * P);
    if (!e && s->Gp) e = pad_gram_launch(s->G, (uint32_t)p, (uint32_t)P, s->Gp, s->stream);
    if (!e) e = hipStreamSynchronize(s->stream);
    if (cm) (void)hipFree(cm);
    if (work) (void)hipFree(work);
    if (raw) (void)hipFree(raw);
    HIP_TRY(e);
    {
        Ctrl c;
        HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (c.err & kErrInput)
            return fail(nullptr, HSP_EINVAL,
                        "y must hold only 0/1 and X must be finite (also after bfloat16 rounding)");
    }
    HIP_TRY(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipEventCreateWithFlags(&s->copied[i], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->freed[i], hipEventDisableTiming));
    }
    return chain_impl(s);
}

// The launch descriptions of a streamed sweep in `mode`: one z-pass launch
// per chunk (no p-side group; the chunk's rows, its first global row and its
// device buffer), then the p-side launch, which takes X^T z from the
// accumulator the chunks added into.
hsp_status stream_args(hsp_state* s, uint32_t mode) {
    if (s->sd_mode == mode && s->sdargs) return HSP_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));  // launches in flight read the old ones
    const uint32_t nc = s->nchunks;
    if (!s->sdargs) {
        HIP_TRY(dalloc(&s->sdargs, (size_t)nc + 1));
        HIP_TRY(dalloc(&s->sdtab, (size_t)nc + 1));
        std::vector<const SweepArgs*> tab(nc + 1);
        for (uint32_t i = 0; i <= nc; ++i) tab[i] = s->sdargs + i;
        HIP_TRY(hipMemcpy(s->sdtab, tab.data(), tab.size() * sizeof(SweepArgs*), hipMemcpyHostToDevice));
    }
    s->sd_host.assign(nc + 1, SweepArgs{});
    for (uint32_t c = 0; c < nc; ++c) {
        SweepArgs h = sweep_args(s, kModeZ);
        sweep_finish_args(&h, s->plan);
        const uint32_t r0 = c * s->chunk_rows;
        const uint32_t rows = std::min(s->chunk_rows, s->x.N - r0);
        h.x.X = dev_ptr(static_cast<const void*>(s->stage[c & 1]));
        h.x.N = rows;
        h.first_row = r0;
        h.gp = 0;
        h.idle = 0;
        const uint32_t tiles = (rows + s->plan.rows - 1) / s->plan.rows;
        h.gz = std::max<uint32_t>(1, std::min<uint32_t>(s->plan.gz, (tiles + 3) / 4));
        h.zgroups = (h.gz + kZGroup - 1) / kZGroup;
        s->sd_host[c] = h;
    }
    const uint32_t pmode = (mode & ~kModeZ) | ((mode & kModeZ) ? kModeBsum : 0u);
    SweepArgs h = sweep_args(s, pmode);
    sweep_finish_args(&h, s->plan);
    s->sd_host[nc] = h;
    HIP_TRY(hipMemcpy(s->sdargs, s->sd_host.data(), (nc + 1) * sizeof(SweepArgs), hipMemcpyHostToDevice));
    s->sd_mode = mode;
    return HSP_OK;
}

// One streamed sweep: chunk c is copied into buffer c % 2 on the copy stream
// once the z pass of chunk c - 2 has released it, and its z pass waits for
// the copy; then the p-side launch.
hsp_status enqueue_stream(hsp_state* s, uint32_t mode) {
    hsp_status st = stream_args(s, mode);
    if (st) return st;
    const size_t row_bytes = (size_t)s->x.ld * (s->x.xtype == 0 ? 4 : 2);
    if (mode & kModeZ) {
        for (uint32_t c = 0; c < s->nchunks; ++c) {
            const int slot = c & 1;
            const SweepArgs& h = s->sd_host[c];
            if (s->freed_used[slot]) HIP_TRY(hipStreamWaitEvent(s->copy_stream, s->freed[slot], 0));
            HIP_TRY(hipMemcpyAsync(s->stage[slot], static_cast<const char*>(s->Xhost) + (size_t)h.first_row * row_bytes,
                                   (size_t)h.x.N * row_bytes, hipMemcpyHostToDevice, s->copy_stream));
            HIP_TRY(hipEventRecord(s->copied[slot], s->copy_stream));
            HIP_TRY(hipStreamWaitEvent(s->stream, s->copied[slot], 0));
            HIP_TRY(sweep_launch(h, s->sdtab + c, s->plan, s->stream));
            HIP_TRY(hipEventRecord(s->freed[slot], s->stream));
            s->freed_used[slot] = true;
        }
    }
    HIP_TRY(sweep_launch(s->sd_host[s->nchunks], s->sdtab + s->nchunks, s->plan, s->stream));
    return HSP_OK;
}

// A further chain on the data of `owner` (same X, y, G; its own Markov state,
// draw ring, factorisation buffers and control block).
hsp_status clone_impl(hsp_state* s, const hsp_state* owner) {
    hsp_status st0 = setup_impl(s);
    if (st0) return st0;
    s->owner = owner;
    s->x = owner->x;
    s->Xbuf = owner->Xbuf;
    s->xexp = owner->xexp;
    s->xscale = owner->xscale;
    s->xscale_h = owner->xscale_h;
    s->y = owner->y;
    s->G = owner->G;
    s->Gp = owner->Gp;
    HIP_TRY(dalloc(&s->ctrl, 1));
    HIP_TRY(hipMemsetAsync(s->ctrl, 0, sizeof(Ctrl), s->stream));
    return chain_impl(s);
}

// Everything one chain owns, its launch plan, and the cold start.
hsp_status chain_impl(hsp_state* s) {
    const int64_t N = s->x.N, p = s->x.p;
    const uint32_t ld = s->x.ld;
    // p-sized state
    HIP_TRY(dalloc(&s->beta, p));
    HIP_TRY(dalloc(&s->beta32, ld));
    HIP_TRY(dalloc(&s->lam, p));
    HIP_TRY(dalloc(&s->nu, p));
    HIP_TRY(dalloc(&s->tau, 1));
    HIP_TRY(dalloc(&s->xi, 1));
    HIP_TRY(dalloc(&s->b, p));
    const size_t P = ((size_t)p + kTile - 1) / kTile * kTile;
    if (p > kSmallP) {
        HIP_TRY(dalloc(&s->A, P * P));
        HIP_TRY(dalloc(&s->Linv, P * P));
        HIP_TRY(hipMemsetAsync(s->A, 0, P * P * sizeof(double), s->stream));
        HIP_TRY(hipMemsetAsync(s->Linv, 0, P * P * sizeof(double), s->stream));
    }
    HIP_TRY(dalloc(&s->vec, 2 * (size_t)p + 8));

    HIP_TRY(sweep_plan(s->x, s->num_cus, &s->plan));
    s->plan_note = "built-in";
    if (p > kSmallP) {
        // the factorisation's task lists for the group, and its tile versions
        const uint32_t nt = (uint32_t)(P / kTile);
        // tile versions, then the substitution's 2 nt row flags (p > kSubstP)
        HIP_TRY(dalloc(&s->ver, 2 * (size_t)nt * nt + 2 * (size_t)nt));
        HIP_TRY(hipMemsetAsync(s->ver, 0, (2 * (size_t)nt * nt + 2 * (size_t)nt) * 4, s->stream));
        hsp_status st = upload_schedule(s);
        if (st) return st;
    }
    // z-pass partials and group counters for the largest split any plan uses
    const size_t gz_cap = (size_t)s->plan.capacity;
    HIP_TRY(dalloc(&s->partial, gz_cap * ld));
    {
        const size_t ng = (gz_cap + kZGroup - 1) / kZGroup;
        HIP_TRY(dalloc(&s->bsum, ld));
        HIP_TRY(hipMemsetAsync(s->bsum, 0, ld * sizeof(double), s->stream));
        HIP_TRY(dalloc(&s->zgrp_count, ng));
        HIP_TRY(hipMemsetAsync(s->zgrp_count, 0, ng * sizeof(uint32_t), s->stream));
    }

    if (s->opt.debug_store_z) {
        HIP_TRY(dalloc(&s->zdbg, (size_t)N));
        HIP_TRY(dalloc(&s->adbg, (size_t)N));
        HIP_TRY(hipMemsetAsync(s->zdbg, 0, (size_t)N * sizeof(float), s->stream));
        HIP_TRY(hipMemsetAsync(s->adbg, 0, (size_t)N * sizeof(int32_t), s->stream));
    }
    const size_t cap = (size_t)s->opt.max_draws;
    HIP_TRY(dalloc(&s->ring_beta, cap * p));
    HIP_TRY(dalloc(&s->ring_tau, cap));
    if (s->opt.record_lambda) HIP_TRY(dalloc(&s->ring_lam, cap * p));

    HIP_TRY(dalloc(&s->dargs, 2));
    HIP_TRY(dalloc(&s->dtab, 2));
    {
        const SweepArgs* tab[2] = {s->dargs, s->dargs + 1};
        HIP_TRY(hipMemcpy(s->dtab, tab, sizeof tab, hipMemcpyHostToDevice));
    }
    {
        SweepArgs h;
        HIP_TRY(put_args(s, kModeSweep, 0, &h));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    // cold start (Section 6.1)
    std::vector<double> zeros(p, 0.0), ones(p, 1.0);
    hsp_status st = upload_state(s, zeros.data(), ones.data(), ones.data(), 1.0, 1.0);
    if (st) return st;
    st = set_counters(s, 0);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->streamed) {
        s->plan_note = "streamed (built-in)";
        return HSP_OK;
    }
    if (s->opt.autotune && !s->in_batch) return tune_impl(s);
    return HSP_OK;
}

bool finite_nonneg(const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i]) || v[i] < 0.0) return false;
    return true;
}

}  // namespace

extern "C" {

void hsp_default_options(hsp_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->seed = 1;
    o->chain_id = 0;
    o->x_type = HSP_X_F32;
    o->x_on_host = 0;
    o->record_lambda = 0;
    o->thin = 1;
    o->max_draws = 1024;
    o->hip_stream = nullptr;
    o->debug_store_z = 0;
    o->use_graph = 1;
    o->multi_chain_z = 1;
    o->autotune = 0;
}

int64_t hsp_max_p(void) { return kMaxP; }

hsp_status hsp_create(const float* X, const uint8_t* y, int64_t N, int64_t p,
                      const hsp_options* opt, hsp_state** out) {
    if (!out) return fail(nullptr, HSP_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!X || !y) return fail(nullptr, HSP_EINVAL, "X and y must not be NULL");
    if (N < 2) return fail(nullptr, HSP_EINVAL, "N must be at least 2");
    if (p < 2) return fail(nullptr, HSP_EINVAL, "p must be at least 2");
    if (N >= (int64_t(1) << 32) - 64) return fail(nullptr, HSP_EINVAL, "N must be below 2^32");
    if (p > kMaxP) return fail(nullptr, HSP_EINVAL, "p exceeds hsp_max_p()");
    hsp_state* s = new (std::nothrow) hsp_state();
    if (!s) return fail(nullptr, HSP_ENOMEM, "host allocation failed");
    if (opt) s->opt = *opt;
    else hsp_default_options(&s->opt);
    if (s->opt.x_type != HSP_X_F32 && s->opt.x_type != HSP_X_BF16) {
        delete s;
        return fail(nullptr, HSP_EINVAL, "x_type must be HSP_X_F32 or HSP_X_BF16");
    }
    if (s->opt.thin < 1 || s->opt.max_draws < 1 || s->opt.max_draws > (int64_t(1) << 30)) {
        delete s;
        return fail(nullptr, HSP_EINVAL, "thin must be >= 1 and max_draws in [1, 2^30]");
    }
    hsp_status st = s->opt.x_stream ? create_stream_impl(s, X, y, N, p) : create_impl(s, X, y, N, p);
    if (st != HSP_OK) {
        if (!s->err.empty()) g_create_error = s->err;
        free_state(s);
        return st;
    }
    *out = s;
    return HSP_OK;
}

// ---- batches: many chains, one graph launch per sweep ------------------------------
}  // extern "C"

// Chains that share one launch of the sweep kernel: each has its own p-side
// group and z-pass blocks, all resident together.
struct Pack {
    int xtype = 0;
    int chunks = 1;  // 16-byte vectors per lane per row: the largest of the pack's chains
    uint32_t blocks = 0;
    uint32_t waiting = 0;   // blocks that wait on other blocks of the launch (the p-side groups)
    double bytes = 0.0;     // X read per sweep
    int capacity = 0;       // resident blocks of the pack's kernel on the device
    // chains sharing one bfloat16 design: a multi-chain z pass (its own
    // launch, mc_gz blocks) precedes the launch of their p-side groups
    bool mc = false;
    McArgs* dmc = nullptr;          // device copy of the pass's description
    double* mc_partial = nullptr;   // mc_gz x kMcChains x mc_stride(ld)
    uint32_t* mc_count = nullptr;   // group and unit counters
    uint32_t mc_gz = 0, mc_ld = 0;
    std::vector<size_t> chains;             // indices into hsp_batch::chains
    std::vector<uint32_t> gp, gz;           // the pack's blocks per chain
    SweepArgs* dargs = nullptr;             // one launch description per chain (device)
    const SweepArgs** dtab = nullptr;       // pointers to them (device)
    uint16_t* dmap = nullptr;               // block -> chain within the pack (device)
    std::vector<uint32_t*> sched;           // per-chain task lists and bounds for its gp (device)
    // a shared z queue: the chains have no z blocks of their own; `workers`
    // blocks after every p-side group take all their z passes
    bool queue = false;
    uint32_t workers = 0;
    // p-side groups split over two launches (tile path only): a `pre` pack
    // draws lambda, tau, nu, xi and factors Q while the multi-chain pass runs;
    // the multi-chain pack after it (`split`) takes b and draws beta
    bool pre = false, split = false;
    std::vector<uint32_t> home;             // home chain of each worker (pack-local index)
    std::vector<uint32_t> unit_tiles;       // row tiles per unit of each chain
    PackQ* dq = nullptr;                    // the queue's counters (device)
};

struct hsp_batch {
    std::vector<hsp_state*> chains;  // dataset-major; the first chain of each dataset owns its data
    std::vector<Pack> packs;         // how the chains share launches
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipGraphExec_t graph = nullptr;  // every chain's sweep, one after another
    bool timing = false;
    EventTimer timer;  // timed batched sweeps
    std::string err;
    // launch-shape parameters of the packs (the autotuner may change them)
    uint32_t mc_gz = 0;        // blocks of each multi-chain z pass (0: two per compute unit)
    uint32_t bw_pct = 100;     // pack split model: z-pass bandwidth per block, percent of nominal
    uint32_t pack_max = 0;     // most chains per pack (0: as many as the resident blocks allow)
    uint32_t zq_kib = 64;      // packs of row-per-wave chains share one z queue, units of about this
                               // many KiB of X (0: every chain has z blocks of its own)
    bool overlap = true;       // multi-chain passes on a second stream, beside the other packs
    uint32_t pre_gp = 0;       // blocks per chain factoring Q beside the multi-chain pass (0: after it)
    hipStream_t side = nullptr, side2 = nullptr;  // streams of the passes and of the pre packs
    hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr, join3 = nullptr;  // (captured into the graph only)
    bool autotune = false;
    std::string plan_note = "built-in";
};

namespace {

// Release the packs' device buffers and the captured graph.
void free_packs(hsp_batch* b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    for (Pack& pk : b->packs) {
        if (pk.dmc) (void)hipFree(pk.dmc);
        if (pk.mc_partial) (void)hipFree(pk.mc_partial);
        if (pk.mc_count) (void)hipFree(pk.mc_count);
        if (pk.dargs) (void)hipFree(pk.dargs);
        if (pk.dtab) (void)hipFree(pk.dtab);
        if (pk.dmap) (void)hipFree(pk.dmap);
        if (pk.dq) (void)hipFree(pk.dq);
        for (uint32_t* q : pk.sched)
            if (q) (void)hipFree(q);
    }
    b->packs.clear();
}

void free_batch(hsp_batch* b) {
    if (!b) return;
    free_packs(b);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->join2) (void)hipEventDestroy(b->join2);
    if (b->join3) (void)hipEventDestroy(b->join3);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->side2) (void)hipStreamDestroy(b->side2);
    b->timer.reset();
    for (auto it = b->chains.rbegin(); it != b->chains.rend(); ++it) free_state(*it);  // borrowers first
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

hsp_status batch_fail(hsp_batch* b, hsp_status code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

// ---- packing chains into shared launches ------------------------------------
// A cost model of one chain's sweep for a given split of its blocks:
// the z pass moves its X at a share of the HBM bandwidth proportional to its
// blocks; the p-side takes the longer of its critical chain and its tile
// work spread over the group's other blocks (p <= 128: one block).
struct ChainCost {
    double bytes;     // X per sweep
    uint32_t nt;      // 64-wide tiles per side of Q (0: one-block path)
    uint32_t ntasks;  // tile tasks of the factorisation
    uint32_t gp_max, gz_max;
};

double z_time_us(const ChainCost& c, uint32_t gz, double bytes_per_us_per_block) {
    return c.bytes / (gz * bytes_per_us_per_block) + 5.0;
}

double p_time_us(const ChainCost& c, uint32_t gp) {
    if (c.nt == 0) return 60.0;
    const double chain = 22.0 * c.nt, work = 6.0 * c.ntasks / (gp > 1 ? gp - 1 : 1);
    return (gp > 1 ? std::max(chain, work) : chain + work) + 30.0;
}

uint32_t count_tasks(uint32_t nt) {
    uint32_t n = 0;
    for (uint32_t k = 0; k < nt; ++k) {
        const uint32_t m = nt - k - 1;
        n += 1 + m + k + m * (m + 1) / 2 + m * (k + 1);
    }
    return n;
}

// Blocks of a queue pack: one p-side block per chain, and more for the chain
// whose factorisation is predicted to take longest while that outlasts the
// z passes on the remaining worker blocks; the workers' home chains in
// proportion to the chains' bytes of X; each chain's unit of about zq_kib KiB
// of rows (whole row tiles).
void plan_queue_pack(const hsp_batch* b, Pack& pk, const std::vector<ChainCost>& cost, int cap, double bw,
                     int rows) {
    const size_t nc = pk.chains.size();
    pk.queue = true;
    pk.gp.assign(nc, 1);
    pk.gz.assign(nc, 0);
    double bytes = 0.0;
    for (size_t j = 0; j < nc; ++j) bytes += cost[pk.chains[j]].bytes;
    uint32_t used = (uint32_t)nc;
    while (used + 1 < (uint32_t)cap) {
        const double tz = bytes / ((double)(cap - used) * bw);
        size_t worst = nc;
        double tw = -1.0;
        for (size_t j = 0; j < nc; ++j) {
            const ChainCost& c = cost[pk.chains[j]];
            const double tp = p_time_us(c, pk.gp[j]);
            if (pk.gp[j] < c.gp_max && tp > tw) {
                tw = tp;
                worst = j;
            }
        }
        if (worst == nc || tw <= tz) break;
        ++pk.gp[worst];
        ++used;
    }
    pk.workers = (uint32_t)cap - used;
    pk.blocks = (uint32_t)cap;
    pk.home.resize(pk.workers);
    double acc = 0.0;
    size_t j = 0;
    for (uint32_t w = 0; w < pk.workers; ++w) {
        const double at = (w + 0.5) * bytes / pk.workers;
        while (j + 1 < nc && acc + cost[pk.chains[j]].bytes <= at) acc += cost[pk.chains[j++]].bytes;
        pk.home[w] = (uint32_t)j;
    }
    pk.unit_tiles.resize(nc);
    for (size_t i = 0; i < nc; ++i) {
        const hsp_state* s = b->chains[pk.chains[i]];
        const double tile_bytes = (double)rows * s->x.ld * (s->x.xtype == 0 ? 4 : 2);
        const double want = std::ceil(b->zq_kib * 1024.0 / tile_bytes);
        pk.unit_tiles[i] = (uint32_t)std::min<double>(kZUnitMax, std::max(1.0, want));
    }
}

// Split the chains into packs that fit the device's resident capacity, and
// split each pack's blocks among its chains so that the slowest chain of the
// pack is as fast as the model allows.  A pack holds chains of one storage
// type and one z-pass tile height R (rows per wave tile): the pack's kernel
// is built for its widest rows, and a wider kernel of the same R sums every
// tile of a narrower chain exactly as that chain's own kernel does (its extra
// columns are zeros), so a chain draws in a pack what it draws alone.  Rows
// split over a block's waves are packed only with rows of the same split.
hsp_status plan_packs(hsp_batch* b) {
    const int num_cus = b->chains[0]->num_cus;
    std::vector<bool> taken(b->chains.size(), false);
    // Chains that share a bfloat16 design (at least two, rows of at most
    // kMcMaxLd elements) run the multi-chain z pass, up to kMcChains at a time.
    if (b->chains[0]->opt.multi_chain_z) {
        for (size_t i = 0; i < b->chains.size(); ++i) {
            const hsp_state* own = b->chains[i];
            if (own->owner || own->x.xtype != HSP_X_BF16 || own->x.ld > kMcMaxLd) continue;
            std::vector<size_t> same;
            for (size_t j = 0; j < b->chains.size(); ++j)
                if (j == i || b->chains[j]->owner == own) same.push_back(j);
            if (same.size() < 2) continue;
            for (size_t g0 = 0; g0 < same.size(); g0 += kMcChains) {
                Pack pk;
                pk.xtype = HSP_X_BF16;
                pk.chunks = own->plan.chunks;
                pk.mc = true;
                pk.mc_ld = own->x.ld;
                // one block per claimed unit at most, two per compute unit
                const uint32_t units = ((own->x.N + kMcRows - 1) / kMcRows + kMcUnit - 1) / kMcUnit;
                const uint32_t want = b->mc_gz ? b->mc_gz : 2u * (uint32_t)num_cus;
                pk.mc_gz = std::max<uint32_t>(1, std::min<uint32_t>(want, units));
                for (size_t j = g0; j < std::min(same.size(), g0 + kMcChains); ++j) {
                    pk.chains.push_back(same[j]);
                    taken[same[j]] = true;
                }
                // the p-side groups share the launch that follows the pass
                const int cap = pack_capacity(HSP_X_BF16, pk.chunks, num_cus);
                if (cap < (int)pk.chains.size()) return batch_fail(b, HSP_EHIP, "no resident capacity for a pack");
                const uint32_t nt = own->x.p > (uint32_t)kSmallP ? (own->x.p + kTile - 1) / kTile : 0;
                const uint32_t gmax = nt ? std::min<uint32_t>(kMaxGroup, nt * (nt + 1) / 2) : 1;
                const uint32_t each = std::max<uint32_t>(1, std::min<uint32_t>(gmax, cap / pk.chains.size()));
                pk.gp.assign(pk.chains.size(), each);
                pk.gz.assign(pk.chains.size(), 0);
                pk.blocks = each * (uint32_t)pk.chains.size();
                if (b->pre_gp && nt) {
                    // the factorisations go beside the pass, in a launch of their own
                    Pack pre;
                    pre.xtype = HSP_X_BF16;
                    pre.chunks = pk.chunks;
                    pre.pre = true;
                    pre.chains = pk.chains;
                    const uint32_t g = std::max<uint32_t>(
                        1, std::min<uint32_t>({gmax, b->pre_gp, (uint32_t)cap / 2 / (uint32_t)pk.chains.size()}));
                    pre.gp.assign(pk.chains.size(), g);
                    pre.gz.assign(pk.chains.size(), 0);
                    pre.blocks = g * (uint32_t)pk.chains.size();
                    pk.split = true;
                    b->packs.push_back(std::move(pre));
                }
                b->packs.push_back(std::move(pk));
            }
        }
    }
    // Packs by (storage type, tile height R, and for rows split over the
    // waves the exact split): the row sums of a wide row depend on where the
    // waves' quarters start.
    auto key_of = [&](size_t i) {
        const hsp_state* c = b->chains[i];
        const int xt = c->x.xtype, kc = c->plan.chunks;
        return std::array<int, 3>{xt, rows_for(xt, kc), wide_chunks(xt, kc) ? kc : 0};
    };
    std::vector<std::array<int, 3>> keys;
    for (size_t i = 0; i < b->chains.size(); ++i)
        if (!taken[i] && std::find(keys.begin(), keys.end(), key_of(i)) == keys.end()) keys.push_back(key_of(i));
    std::sort(keys.begin(), keys.end());
    for (const auto& key : keys) {
        const int xt = key[0];
        std::vector<size_t> ids;
        int chunks = 1;
        for (size_t i = 0; i < b->chains.size(); ++i)
            if (!taken[i] && key_of(i) == key) {
                ids.push_back(i);
                chunks = std::max(chunks, b->chains[i]->plan.chunks);
            }
        if (ids.empty()) continue;
        const int cap = pack_capacity(xt, chunks, num_cus);
        if (cap < 2) return batch_fail(b, HSP_EHIP, "no resident capacity for a pack");
        // bytes per microsecond per block (about 7 TB/s in all, scaled by the tuner)
        const double bw = 7.0e6 / cap * (b->bw_pct / 100.0);
        std::vector<ChainCost> cost(b->chains.size());
        const int rows = rows_for(xt, chunks);
        for (size_t i : ids) {
            const hsp_state* s = b->chains[i];
            ChainCost& c = cost[i];
            c.bytes = (double)s->x.N * s->x.ld * (xt == 0 ? 4 : 2);
            c.nt = s->x.p > (uint32_t)kSmallP ? (s->x.p + kTile - 1) / kTile : 0;
            c.ntasks = c.nt ? count_tasks(c.nt) : 0;
            c.gp_max = c.nt ? std::min<uint32_t>(kMaxGroup, c.nt * (c.nt + 1) / 2) : 1;
            const uint32_t tiles = (s->x.N + rows - 1) / rows;
            c.gz_max = std::max<uint32_t>(1, std::min<uint32_t>(s->plan.gz, (tiles + 3) / 4));
        }
        std::sort(ids.begin(), ids.end(), [&](size_t x, size_t y) { return cost[x].bytes > cost[y].bytes; });
        // packs of at most cap blocks, two blocks per chain at least
        std::vector<std::vector<size_t>> groups;
        for (size_t i : ids) {
            if (groups.empty() || 2 * (groups.back().size() + 1) > (size_t)cap ||
                (b->pack_max && groups.back().size() >= b->pack_max))
                groups.emplace_back();
            groups.back().push_back(i);
        }
        const bool queue = b->zq_kib > 0 && key[2] == 0;
        for (auto& g : groups) {
            Pack pk;
            pk.xtype = xt;
            pk.chunks = chunks;
            pk.chains = g;
            if (queue && g.size() <= (size_t)kPackQMax) {
                plan_queue_pack(b, pk, cost, cap, bw, rows);
                b->packs.push_back(std::move(pk));
                continue;
            }
            pk.gp.assign(g.size(), 1);
            pk.gz.assign(g.size(), 1);
            uint32_t used = 2 * (uint32_t)g.size();
            while (used < (uint32_t)cap) {
                // the chain predicted to finish last gets one more block where it helps
                size_t worst = g.size();
                double tw = -1.0;
                bool to_z = true;
                for (size_t j = 0; j < g.size(); ++j) {
                    const ChainCost& c = cost[g[j]];
                    const double tz = z_time_us(c, pk.gz[j], bw), tp = p_time_us(c, pk.gp[j]);
                    const bool can_z = pk.gz[j] < c.gz_max, can_p = pk.gp[j] < c.gp_max;
                    const bool zj = tz >= tp ? can_z : !can_p;
                    if (!(zj ? can_z : can_p)) continue;
                    const double t = std::max(tz, tp);
                    if (t > tw) {
                        tw = t;
                        worst = j;
                        to_z = zj;
                    }
                }
                if (worst == g.size()) break;
                if (to_z) ++pk.gz[worst];
                else ++pk.gp[worst];
                ++used;
            }
            pk.blocks = used;
            b->packs.push_back(std::move(pk));
        }
    }
    // device descriptions, block maps and schedules
    for (Pack& pk : b->packs) {
        const size_t nc = pk.chains.size();
        if (dalloc(&pk.dargs, nc) || dalloc(&pk.dtab, nc) || dalloc(&pk.dmap, pk.blocks))
            return batch_fail(b, HSP_ENOMEM, "pack allocation failed");
        std::vector<SweepArgs> host(nc);
        std::vector<const SweepArgs*> tab(nc);
        std::vector<uint16_t> map(pk.blocks);
        PackQ hq{};
        if (pk.queue) {
            if (dalloc(&pk.dq, 1)) return batch_fail(b, HSP_ENOMEM, "pack allocation failed");
            hq.nchains = (uint32_t)nc;
            hq.workers = pk.workers;
        }
        uint32_t blk = 0;
        for (size_t j = 0; j < nc; ++j) {
            hsp_state* s = b->chains[pk.chains[j]];
            // a chain of a multi-chain pack takes b from the pass before; a
            // pre pack's launch stops where b is needed, and the split pack's
            // launch starts there
            uint32_t mode = pk.mc ? (kModeSweep & ~kModeZ) | kModeBsum : kModeSweep;
            if (pk.pre) mode = kModeLambda | kModeTau | kModeNuXi | kModeBeta | kModePre;
            else if (pk.split) mode = kModeBeta | kModeRecord | kModeAdvance | kModeBsum | kModePost;
            SweepArgs h = sweep_args(s, mode);
            h.gp = pk.gp[j];
            h.gz = pk.gz[j];
            h.z_static_pct = kZStaticPctDefault;
            h.z_unit = kZUnitDefault;
            h.zgroups = (h.gz + kZGroup - 1) / kZGroup;
            if (pk.queue) {
                // the p-side waits for the chain's units instead of its groups
                const uint32_t tiles = (s->x.N + rows_for(pk.xtype, pk.chunks) - 1) / rows_for(pk.xtype, pk.chunks);
                h.z_unit = pk.unit_tiles[j];
                hq.units[j] = (tiles + h.z_unit - 1) / h.z_unit;
                h.zgroups = hq.units[j];
                h.zq = dev_ptr(pk.dq);
            }
            h.block0 = blk;
            // the chains of a multi-chain pass factor Q beside or after the
            // pass, not under a pass of their own: there the factorisation
            // without L^-1 (half the tile tasks and their traffic) and beta
            // by substitution take less time than the inverse and the two
            // products (they already round differently from a lone chain)
            if ((pk.mc || pk.pre || pk.split) && s->x.p > (uint32_t)kSmallP) h.subst = 1u;
            if (s->x.p > (uint32_t)kSmallP && !pk.split) {
                const uint32_t nt = (s->x.p + kTile - 1) / kTile;
                std::vector<uint32_t> tasks, off;
                chol_schedule(nt, h.gp, &tasks, &off, h.subst == 0u);
                uint32_t *dt = nullptr, *doff = nullptr;
                if (dalloc(&dt, tasks.size()) || dalloc(&doff, off.size()))
                    return batch_fail(b, HSP_ENOMEM, "pack allocation failed");
                pk.sched.push_back(dt);
                pk.sched.push_back(doff);
                if (hipMemcpy(dt, tasks.data(), tasks.size() * 4, hipMemcpyHostToDevice) ||
                    hipMemcpy(doff, off.data(), off.size() * 4, hipMemcpyHostToDevice))
                    return batch_fail(b, HSP_EHIP, "pack schedule upload");
                h.tasks = dev_ptr(static_cast<const uint32_t*>(dt));
                h.task_off = dev_ptr(static_cast<const uint32_t*>(doff));
            }
            host[j] = h;
            tab[j] = pk.dargs + j;
            for (uint32_t q = 0; q < h.gp + h.gz; ++q) map[blk + q] = (uint16_t)j;
            blk += h.gp + h.gz;
        }
        pk.waiting = 0;
        pk.bytes = 0.0;
        for (size_t j = 0; j < nc; ++j) {
            const hsp_state* s = b->chains[pk.chains[j]];
            pk.waiting += pk.gp[j];
            if (!pk.pre) pk.bytes += (double)s->x.N * s->x.ld * (s->x.xtype == 0 ? 4 : 2);
        }
        pk.capacity = pack_capacity(pk.xtype, pk.chunks, b->chains[0]->num_cus);
        if (pk.queue) {
            // the workers follow every p-side group
            for (uint32_t w = 0; w < pk.workers; ++w) map[blk + w] = (uint16_t)(kWorkerBit | pk.home[w]);
            blk += pk.workers;
            if (hipMemcpy(pk.dq, &hq, sizeof hq, hipMemcpyHostToDevice))
                return batch_fail(b, HSP_EHIP, "pack upload");
        }
        if (blk != pk.blocks) return batch_fail(b, HSP_EHIP, "pack block map does not cover the launch");
        if (hipMemcpy(pk.dargs, host.data(), nc * sizeof(SweepArgs), hipMemcpyHostToDevice) ||
            hipMemcpy(pk.dtab, tab.data(), nc * sizeof(const SweepArgs*), hipMemcpyHostToDevice) ||
            hipMemcpy(pk.dmap, map.data(), map.size() * 2, hipMemcpyHostToDevice))
            return batch_fail(b, HSP_EHIP, "pack upload");
        if (pk.mc) {
            const hsp_state* own = b->chains[pk.chains[0]];
            McArgs m{};
            m.x = own->x;
            m.y = dev_ptr(static_cast<const uint8_t*>(own->y));
            m.nchains = (uint32_t)nc;
            m.gz = pk.mc_gz;
            m.zgroups = (m.gz + kZGroup - 1) / kZGroup;
            const size_t ncount = (size_t)m.zgroups + 64;
            m.pstride = mc_stride(pk.mc_ld);
            if (dalloc(&pk.dmc, 1) || dalloc(&pk.mc_partial, (size_t)m.gz * kMcChains * m.pstride) ||
                dalloc(&pk.mc_count, ncount))
                return batch_fail(b, HSP_ENOMEM, "pack allocation failed");
            m.partial = dev_ptr(pk.mc_partial);
            m.count = dev_ptr(pk.mc_count);
            for (size_t j = 0; j < nc; ++j) m.chain[j] = dev_ptr(static_cast<const SweepArgs*>(pk.dargs + j));
            if (hipMemset(pk.mc_count, 0, ncount * 4) || hipMemcpy(pk.dmc, &m, sizeof m, hipMemcpyHostToDevice))
                return batch_fail(b, HSP_EHIP, "pack upload");
        }
    }
    return HSP_OK;
}

// The packs (if not planned yet) and the graph of one batched sweep.
hsp_status batch_build(hsp_batch* b) {
    if (b->packs.empty()) {
        hsp_status st = plan_packs(b);
        if (st != HSP_OK) return st;
    }
    if (b->graph) return HSP_OK;
    bool any_mc = false, any_pre = false;
    size_t n_plain = 0;
    for (const Pack& pk : b->packs) {
        if (pk.pre) any_pre = true;
        else if (pk.mc) any_mc = true;
        else ++n_plain;
    }
    const bool overlap = b->overlap && ((any_mc && (n_plain > 0 || any_pre)) || n_plain > 1);
    hipError_t e = hipSuccess;
    if (overlap && !b->side) {
        e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (!e) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (!e) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (!e) e = hipEventCreateWithFlags(&b->join3, hipEventDisableTiming);
        if (e) return batch_fail(b, HSP_EHIP, std::string("batch side stream: ") + hipGetErrorString(e));
    }
    if (overlap && any_pre && !b->side2) {
        e = hipStreamCreateWithFlags(&b->side2, hipStreamNonBlocking);
        if (!e) e = hipEventCreateWithFlags(&b->join2, hipEventDisableTiming);
        if (e) return batch_fail(b, HSP_EHIP, std::string("batch side stream: ") + hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    auto launch = [&](const Pack& pk, hipStream_t st) {
        return pack_launch(pk.xtype, pk.chunks, pk.dtab, pk.dmap, pk.blocks, st);
    };
    if (overlap) {
        // The multi-chain passes, and the pre packs (whose blocks wait only
        // on blocks of their own launch), may run beside the other packs, on
        // streams of their own; blocks of one launch become resident as
        // blocks of another finish.  The launches that take b from a pass
        // follow them on the batch's stream.
        if (!e) e = hipEventRecord(b->fork, b->stream);
        if (!e) e = hipStreamWaitEvent(b->side, b->fork, 0);
        for (size_t i = 0; !e && i < b->packs.size(); ++i)
            if (b->packs[i].mc) e = mc_launch(b->packs[i].dmc, b->packs[i].mc_ld, b->packs[i].mc_gz, b->side);
        if (!e) e = hipEventRecord(b->join, b->side);
        if (any_pre) {
            if (!e) e = hipStreamWaitEvent(b->side2, b->fork, 0);
            for (size_t i = 0; !e && i < b->packs.size(); ++i)
                if (b->packs[i].pre) e = launch(b->packs[i], b->side2);
            if (!e) e = hipEventRecord(b->join2, b->side2);
        }
        // The other packs: the one with the most X on the batch's stream, the
        // rest after the passes on theirs, if every launch that may then be
        // resident at once leaves at least half of the device to blocks that
        // never wait.
        std::vector<size_t> plain;
        int waiting = 0, cap = 0;
        for (size_t i = 0; i < b->packs.size(); ++i) {
            const Pack& pk = b->packs[i];
            if (!pk.mc) waiting += (int)pk.waiting;  // pre packs wait inside too
            if (!pk.mc && !pk.pre) plain.push_back(i);
            cap = cap ? std::min(cap, pk.capacity) : pk.capacity;
        }
        std::stable_sort(plain.begin(), plain.end(),
                         [&](size_t x, size_t y) { return b->packs[x].bytes > b->packs[y].bytes; });
        const bool spread = plain.size() > 1 && 2 * waiting <= cap;
        for (size_t k = 0; !e && k < plain.size(); ++k)
            e = launch(b->packs[plain[k]], spread && k > 0 ? b->side : b->stream);
        if (!e && spread) e = hipEventRecord(b->join3, b->side);
        if (!e) e = hipStreamWaitEvent(b->stream, b->join, 0);
        if (!e && any_pre) e = hipStreamWaitEvent(b->stream, b->join2, 0);
        for (size_t i = 0; !e && i < b->packs.size(); ++i)
            if (b->packs[i].mc) e = launch(b->packs[i], b->stream);
        if (!e && spread) e = hipStreamWaitEvent(b->stream, b->join3, 0);
    } else {
        // in pack order: a pre pack comes just before its multi-chain pack
        for (size_t i = 0; !e && i < b->packs.size(); ++i) {
            const Pack& pk = b->packs[i];
            if (pk.mc) e = mc_launch(pk.dmc, pk.mc_ld, pk.mc_gz, b->stream);
            if (!e) e = launch(pk, b->stream);
        }
    }
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (!e) e = e2;
    if (!e) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e) return batch_fail(b, HSP_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e));
    return HSP_OK;
}

// Cache key of a batch: the device and a hash of every chain's design.
std::string batch_tune_key(const hsp_batch* b) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the batch's description
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)b->chains[0]->opt.multi_chain_z);
    for (size_t i = 0; i < b->chains.size(); ++i) {
        const hsp_state* s = b->chains[i];
        mix(s->x.N);
        mix(s->x.p);
        mix((uint64_t)s->x.xtype);
        size_t own = i;
        for (size_t j = 0; j < b->chains.size(); ++j)
            if (b->chains[j] == (s->owner ? s->owner : s)) own = j;
        mix(own);
    }
    char hex[17];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)h);
    const hsp_state* s0 = b->chains[0];
    return "batch-v6 " + device_tag(s0->device, s0->num_cus) + " chains=" + std::to_string(b->chains.size()) +
           " h=" + hex;
}

// Mean milliseconds of `timed` replays of the batch's graph after `warm`.
hsp_status time_batch(hsp_batch* b, int warm, int timed, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return batch_fail(b, HSP_EHIP, "event");
    hipError_t e = hipEventCreate(&e1);
    for (int i = 0; !e && i < warm; ++i) e = hipGraphLaunch(b->graph, b->stream);
    if (!e) e = hipEventRecord(e0, b->stream);
    for (int i = 0; !e && i < timed; ++i) e = hipGraphLaunch(b->graph, b->stream);
    if (!e) e = hipEventRecord(e1, b->stream);
    if (!e) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (!e) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e) return batch_fail(b, HSP_EHIP, std::string("timing a batched sweep: ") + hipGetErrorString(e));
    *ms = (double)t / timed;
    for (size_t i = 0; i < b->chains.size(); ++i) {
        hsp_status st = check_device_flags(b->chains[i]);
        if (st != HSP_OK) return batch_fail(b, st, "chain " + std::to_string(i) + ": " + b->chains[i]->err);
    }
    return HSP_OK;
}

// The autotuner for a batch: blocks of each multi-chain z pass, chains per
// pack, the bandwidth the pack split model gives a z-pass block, whether the
// packs share one z queue (and its unit size), how many blocks per chain
// factor Q beside the multi-chain pass, and whether the passes run beside
// the other packs, by timing a few batched sweeps of every candidate (or
// from the cache).  Every chain's state is put back afterwards.
hsp_status batch_tune(hsp_batch* b) {
    const std::string key = batch_tune_key(b);
    const char* path = tune_cache_path();
    std::string cached;
    long mcg = 0, bwp = 0, pmax = 0, ov = 1, zq = 0, pre = 0;
    if (path && tune_cache_get(path, key, &cached) && tune_parse(cached, "mc_gz", &mcg) &&
        tune_parse(cached, "bw", &bwp) && tune_parse(cached, "pack", &pmax) && tune_parse(cached, "ov", &ov) &&
        tune_parse(cached, "zq", &zq) && tune_parse(cached, "pre", &pre) && mcg >= 0 && mcg <= 65536 &&
        bwp >= 10 && bwp <= 1000 && pmax >= 0 && pmax <= 65536 && (ov == 0 || ov == 1) && zq >= 0 &&
        zq <= 4096 && pre >= 0 && pre <= 4096) {
        b->mc_gz = (uint32_t)mcg;
        b->bw_pct = (uint32_t)bwp;
        b->pack_max = (uint32_t)pmax;
        b->overlap = ov != 0;
        b->zq_kib = (uint32_t)zq;
        b->pre_gp = (uint32_t)pre;
        b->plan_note = "mc_gz=" + std::to_string(mcg) + " bw=" + std::to_string(bwp) + " pack=" +
                       std::to_string(pmax) + " ov=" + std::to_string(ov) + " zq=" + std::to_string(zq) +
                       " pre=" + std::to_string(pre) + " (cache)";
        return HSP_OK;
    }
    std::vector<SavedChain> saved(b->chains.size());
    for (size_t i = 0; i < b->chains.size(); ++i) {
        hsp_status st = save_chain(b->chains[i], &saved[i]);
        if (st) return batch_fail(b, st, b->chains[i]->err);
    }
    // is there a multi-chain pass to size?
    hsp_status st = plan_packs(b);
    if (st) return st;
    uint32_t units = 0;
    for (const Pack& pk : b->packs)
        if (pk.mc) {
            const hsp_state* own = b->chains[pk.chains[0]];
            units = std::max(units, ((own->x.N + kMcRows - 1) / kMcRows + kMcUnit - 1) / kMcUnit);
        }
    free_packs(b);
    const uint32_t cus = (uint32_t)b->chains[0]->num_cus;
    std::vector<uint32_t> mcs{0};
    if (units)
        for (uint32_t m : {cus / 2, cus, 3 * cus / 2, 2 * cus, 3 * cus})
            if (m >= 1 && m <= units && std::find(mcs.begin(), mcs.end(), m) == mcs.end()) mcs.push_back(m);
    // chains per pack: all that fit, or fewer chains each with more blocks
    std::vector<uint32_t> pmaxs{0};
    for (uint32_t m : {32u, 16u, 8u, 4u})
        if (m < b->chains.size()) pmaxs.push_back(m);
    double best_ms = 1e300;
    uint32_t best_mc = 0, best_bw = 100, best_pm = 0, best_zq = 0;
    // every candidate is timed over a few replays; the best few are timed
    // again over more (the least of many short, noisy timings favours
    // whichever candidate was lucky)
    struct Cand {
        double ms;
        uint32_t mc, bw, pm, zq;
    };
    std::vector<Cand> cands;
    auto trial = [&](uint32_t pm, uint32_t mc, uint32_t bw, uint32_t zq) -> hsp_status {
        b->mc_gz = mc;
        b->bw_pct = bw;
        b->pack_max = pm;
        b->zq_kib = zq;
        hsp_status s2 = batch_build(b);
        double ms = 0.0;
        if (!s2) s2 = time_batch(b, 1, 3, &ms);
        free_packs(b);
        if (s2) return s2;
        cands.push_back(Cand{ms, mc, bw, pm, zq});
        if (ms < best_ms) {
            best_ms = ms;
            best_mc = mc;
            best_bw = bw;
            best_pm = pm;
            best_zq = zq;
        }
        return HSP_OK;
    };
    constexpr int kLongWarm = 2, kLongTimed = 12;
    // a shared z queue per pack: its unit size, blocks per multi-chain pass
    // and chains per pack
    for (uint32_t zq : {32u, 64u, 128u})
        for (uint32_t mc : mcs)
            for (uint32_t pm : {0u, 32u})
                if ((pm == 0 || pm < b->chains.size()) && (st = trial(pm, mc, 100, zq)) != HSP_OK) return st;
    // chains with z blocks of their own: chains per pack and the split
    // model's bandwidth, with the best pass size so far or the built-in one
    std::vector<uint32_t> mc_c{best_mc};
    if (best_mc != 0) mc_c.push_back(0);
    for (uint32_t mc : mc_c)
        for (uint32_t pm : pmaxs)
            for (uint32_t bw : {60u, 100u, 160u})
                if ((st = trial(pm, mc, bw, 0)) != HSP_OK) return st;
    {
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        best_ms = 1e300;
        for (size_t i = 0; i < cands.size() && i < 3; ++i) {
            const Cand& c = cands[i];
            b->mc_gz = c.mc;
            b->bw_pct = c.bw;
            b->pack_max = c.pm;
            b->zq_kib = c.zq;
            st = batch_build(b);
            double ms = 0.0;
            if (!st) st = time_batch(b, kLongWarm, kLongTimed, &ms);
            free_packs(b);
            if (st) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best_mc = c.mc;
                best_bw = c.bw;
                best_pm = c.pm;
                best_zq = c.zq;
            }
        }
    }
    b->mc_gz = best_mc;
    b->bw_pct = best_bw;
    b->pack_max = best_pm;
    b->zq_kib = best_zq;
    uint32_t best_pre = b->pre_gp;
    if (units) {
        // blocks per chain factoring Q beside the multi-chain pass (0: after it)
        const uint32_t tried = b->pre_gp;
        for (uint32_t pg : {0u, 8u, 32u}) {
            if (pg == tried) continue;
            b->pre_gp = pg;
            st = batch_build(b);
            double ms = 0.0;
            if (!st) st = time_batch(b, kLongWarm, kLongTimed, &ms);
            free_packs(b);
            if (st) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best_pre = pg;
            }
        }
        b->pre_gp = best_pre;
    }
    bool best_ov = true;
    {
        // the passes beside the packs, or all launches one after another
        b->overlap = false;
        st = batch_build(b);
        double ms = 0.0;
        if (!st) st = time_batch(b, kLongWarm, kLongTimed, &ms);
        free_packs(b);
        if (st) return st;
        if (ms < best_ms) {
            best_ms = ms;
            best_ov = false;
        }
        b->overlap = best_ov;
    }
    for (size_t i = 0; i < b->chains.size(); ++i) {
        st = restore_chain(b->chains[i], saved[i]);
        if (st) return batch_fail(b, st, b->chains[i]->err);
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "mc_gz=%u bw=%u pack=%u ov=%d zq=%u pre=%u ms=%.4f", best_mc, best_bw, best_pm,
                  (int)best_ov, best_zq, best_pre, best_ms);
    b->plan_note = std::string(buf) + " (measured)";
    if (path) (void)tune_cache_put(path, key, buf);
    return HSP_OK;
}

}  // namespace

extern "C" {

hsp_status hsp_batch_create(const hsp_dataset* ds, int32_t n_ds, const int32_t* chains_per_ds,
                            const hsp_options* opt, hsp_batch** out) {
    if (!out) return fail(nullptr, HSP_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!ds || !chains_per_ds || n_ds < 1) return fail(nullptr, HSP_EINVAL, "bad batch description");
    hsp_options base;
    if (opt) base = *opt;
    else hsp_default_options(&base);
    int64_t total = 0;
    for (int32_t d = 0; d < n_ds; ++d) {
        if (chains_per_ds[d] < 1) return fail(nullptr, HSP_EINVAL, "every dataset needs at least one chain");
        total += chains_per_ds[d];
    }
    if (total > 65536) return fail(nullptr, HSP_EINVAL, "at most 65536 chains per batch");
    hsp_batch* b = new (std::nothrow) hsp_batch();
    if (!b) return fail(nullptr, HSP_ENOMEM, "host allocation failed");
    if (base.hip_stream) {
        b->stream = static_cast<hipStream_t>(base.hip_stream);
    } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(nullptr, HSP_EHIP, "stream creation failed");
    }
    else {
        b->own_stream = true;
    }
    uint32_t chain_id = base.chain_id;
    for (int32_t d = 0; d < n_ds; ++d) {
        hsp_state* owner = nullptr;
        for (int32_t c = 0; c < chains_per_ds[d]; ++c, ++chain_id) {
            hsp_options o = base;
            o.hip_stream = b->stream;
            o.x_type = ds[d].x_type;
            o.chain_id = chain_id;
            o.use_graph = 1;
            o.autotune = 0;  // the batch tunes its packs instead
            o.x_stream = 0;  // every dataset of a batch is resident
            hsp_state* s = nullptr;
            hsp_status st;
            if (c == 0) {
                st = hsp_create(ds[d].X, ds[d].y, ds[d].N, ds[d].p, &o, &s);
            } else {
                s = new (std::nothrow) hsp_state();
                if (!s) {
                    st = fail(nullptr, HSP_ENOMEM, "host allocation failed");
                } else {
                    s->opt = o;
                    st = clone_impl(s, owner);
                    if (st != HSP_OK) {
                        if (!s->err.empty()) g_create_error = s->err;
                        free_state(s);
                        s = nullptr;
                    }
                }
            }
            if (st != HSP_OK) {
                free_batch(b);
                return st;
            }
            s->in_batch = true;
            if (c == 0) owner = s;
            b->chains.push_back(s);
        }
    }
    b->autotune = base.autotune != 0;
    *out = b;
    return HSP_OK;
}

int64_t hsp_batch_size(const hsp_batch* b) { return b ? (int64_t)b->chains.size() : 0; }

hsp_status hsp_batch_chain(hsp_batch* b, int64_t i, hsp_state** chain) {
    if (!b || !chain || i < 0 || i >= (int64_t)b->chains.size())
        return batch_fail(b, HSP_EINVAL, "chain index out of range");
    *chain = b->chains[(size_t)i];
    return HSP_OK;
}

hsp_status hsp_batch_sweep(hsp_batch* b, int64_t n) {
    if (!b) return HSP_EINVAL;
    if (n < 0) return batch_fail(b, HSP_EINVAL, "n_iter must be >= 0");
    for (hsp_state* s : b->chains) {
        if (s->poisoned) return batch_fail(b, HSP_EPOISONED, "a chain of the batch is poisoned");
        if (s->sweeps_done + (uint64_t)n >= (uint64_t(1) << 32) - 1)
            return batch_fail(b, HSP_EINVAL, "the sweep counter would exceed 2^32");
    }
    if (!b->graph) {
        if (b->autotune) {
            b->autotune = false;  // once per batch
            hsp_status st = batch_tune(b);
            if (st != HSP_OK) return st;
        }
        hsp_status st = batch_build(b);
        if (st != HSP_OK) return st;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (b->timing && b->timer.begin(b->stream) != hipSuccess)
            return batch_fail(b, HSP_EHIP, "timing event");
        if (hipGraphLaunch(b->graph, b->stream) != hipSuccess)
            return batch_fail(b, HSP_EHIP, "batch graph launch");
        if (b->timing && b->timer.end(b->stream) != hipSuccess)
            return batch_fail(b, HSP_EHIP, "timing event");
    }
    for (hsp_state* s : b->chains) s->sweeps_done += (uint64_t)n;
    return HSP_OK;
}

hsp_status hsp_batch_sync(hsp_batch* b) {
    if (!b) return HSP_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return batch_fail(b, HSP_EHIP, "stream synchronisation");
    for (size_t i = 0; i < b->chains.size(); ++i) {
        hsp_status st = check_device_flags(b->chains[i]);
        if (st != HSP_OK) return batch_fail(b, st, "chain " + std::to_string(i) + ": " + b->chains[i]->err);
    }
    return HSP_OK;
}

hsp_status hsp_batch_set_timing(hsp_batch* b, int32_t enable) {
    if (!b) return HSP_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return batch_fail(b, HSP_EHIP, "stream synchronisation");
    b->timer.reset();
    b->timing = enable != 0;
    return HSP_OK;
}

hsp_status hsp_batch_get_timing(hsp_batch* b, double* ms_per_sweep, int64_t* n) {
    if (!b || !ms_per_sweep) return HSP_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return batch_fail(b, HSP_EHIP, "stream synchronisation");
    double span = 0.0;
    int64_t cnt = 0;
    if (b->timer.result(ms_per_sweep, &span, &cnt) != hipSuccess) return batch_fail(b, HSP_EHIP, "event timing");
    if (n) *n = cnt;
    return HSP_OK;
}

const char* hsp_batch_last_error(const hsp_batch* b) {
    return b ? b->err.c_str() : g_create_error.c_str();
}

hsp_status hsp_batch_destroy(hsp_batch* b) {
    if (!b) return HSP_EINVAL;
    free_batch(b);
    return HSP_OK;
}

hsp_status hsp_sweep(hsp_state* s, int64_t n) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    if (n < 0) return fail(s, HSP_EINVAL, "n_iter must be >= 0");
    if (s->sweeps_done + (uint64_t)n >= (uint64_t(1) << 32) - 1)
        return fail(s, HSP_EINVAL, "the sweep counter would exceed 2^32");
    if (s->streamed) {
        for (int64_t i = 0; i < n; ++i) {
            if (s->timing) HIP_TRY(s->timer.begin(s->stream));
            hsp_status st = enqueue_stream(s, kModeSweep);
            if (st) return st;
            if (s->timing) HIP_TRY(s->timer.end(s->stream));
        }
        s->sweeps_done += (uint64_t)n;
        return HSP_OK;
    }
    if (s->opt.use_graph && !s->graph) {
        hipError_t e = capture(s, &s->graph);
        if (e) return fail_hip(s, "graph capture", e);
    }
    for (int64_t i = 0; i < n; ++i) {
        if (s->timing) HIP_TRY(s->timer.begin(s->stream));
        if (s->graph) HIP_TRY(hipGraphLaunch(s->graph, s->stream));
        else HIP_TRY(enqueue_sweep(s, s->stream));
        if (s->timing) HIP_TRY(s->timer.end(s->stream));
    }
    s->sweeps_done += (uint64_t)n;
    return HSP_OK;
}

hsp_status hsp_sync(hsp_state* s) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    return sync_state(s);
}

hsp_status hsp_draws(hsp_state* s, double* beta, double* tau_m2, double* lam_m2, int64_t first,
                     int64_t count, int64_t* n_out) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    hsp_status st = sync_state(s);
    if (st) return st;
    const int64_t recorded = (int64_t)((s->sweeps_done - s->draw_base) / (uint64_t)s->opt.thin);
    if (n_out) *n_out = recorded;
    if (count == 0) return HSP_OK;
    if (first < 0 || count < 0 || first + count > recorded || first < recorded - s->opt.max_draws)
        return fail(s, HSP_EINVAL, "requested draws are not stored (range or overwritten)");
    if (lam_m2 && !s->ring_lam) return fail(s, HSP_EINVAL, "lambda was not recorded");
    const int64_t cap = s->opt.max_draws;
    const size_t p = s->x.p;
    for (int64_t d = first; d < first + count;) {
        const int64_t slot = d % cap;
        const int64_t run = std::min(first + count - d, cap - slot);
        const int64_t o = d - first;
        if (beta)
            HIP_TRY(hipMemcpy(beta + o * p, s->ring_beta + slot * p, run * p * sizeof(double),
                              hipMemcpyDeviceToHost));
        if (tau_m2)
            HIP_TRY(hipMemcpy(tau_m2 + o, s->ring_tau + slot, run * sizeof(double),
                              hipMemcpyDeviceToHost));
        if (lam_m2)
            HIP_TRY(hipMemcpy(lam_m2 + o * p, s->ring_lam + slot * p, run * p * sizeof(double),
                              hipMemcpyDeviceToHost));
        d += run;
    }
    return HSP_OK;
}

hsp_status hsp_destroy(hsp_state* s) {
    if (s && s->in_batch) return fail(s, HSP_EINVAL, "this chain belongs to a batch: destroy the batch");
    free_state(s);
    return HSP_OK;
}

const char* hsp_last_error(const hsp_state* s) {
    if (!s) return g_create_error.c_str();
    return s->err.c_str();
}

hsp_status hsp_get_state(hsp_state* s, double* beta, double* lam_m2, double* nu_m1,
                         double* tau_m2, double* xi_m1, uint64_t* sweep) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    hsp_status st = sync_state(s);
    if (st) return st;
    const size_t p = s->x.p;
    if (beta) HIP_TRY(hipMemcpy(beta, s->beta, p * sizeof(double), hipMemcpyDeviceToHost));
    if (lam_m2) HIP_TRY(hipMemcpy(lam_m2, s->lam, p * sizeof(double), hipMemcpyDeviceToHost));
    if (nu_m1) HIP_TRY(hipMemcpy(nu_m1, s->nu, p * sizeof(double), hipMemcpyDeviceToHost));
    if (tau_m2) HIP_TRY(hipMemcpy(tau_m2, s->tau, sizeof(double), hipMemcpyDeviceToHost));
    if (xi_m1) HIP_TRY(hipMemcpy(xi_m1, s->xi, sizeof(double), hipMemcpyDeviceToHost));
    if (sweep) *sweep = s->sweeps_done;
    return HSP_OK;
}

hsp_status hsp_set_state(hsp_state* s, const double* beta, const double* lam_m2,
                         const double* nu_m1, double tau_m2, double xi_m1, uint64_t sweep) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    if (!beta || !lam_m2 || !nu_m1) return fail(s, HSP_EINVAL, "state vectors must not be NULL");
    const int64_t p = s->x.p;
    for (int64_t j = 0; j < p; ++j)
        if (!std::isfinite(beta[j])) return fail(s, HSP_EINVAL, "beta must be finite");
    if (!finite_nonneg(lam_m2, p) || !finite_nonneg(nu_m1, p) || !finite_nonneg(&tau_m2, 1) ||
        !finite_nonneg(&xi_m1, 1))
        return fail(s, HSP_EINVAL, "lam_m2, nu_m1, tau_m2, xi_m1 must be finite and >= 0");
    if (sweep >= (uint64_t(1) << 32) - 1) return fail(s, HSP_EINVAL, "sweep must be below 2^32");
    HIP_TRY(hipStreamSynchronize(s->stream));
    hsp_status st = upload_state(s, beta, lam_m2, nu_m1, tau_m2, xi_m1);
    if (st) return st;
    return set_counters(s, sweep);
}

hsp_status hsp_step(hsp_state* s, uint32_t which) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    uint32_t mode = 0;
    if (which & HSP_STEP_Z) mode |= kModeZ;
    if (which & HSP_STEP_LAMBDA) mode |= kModeLambda;
    if (which & HSP_STEP_TAU) mode |= kModeTau;
    if (which & HSP_STEP_BETA) mode |= kModeBeta;
    if (which & HSP_STEP_NUXI) mode |= kModeNuXi;
    if (which & HSP_STEP_ADVANCE) mode |= kModeAdvance;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->streamed) {
        hsp_status st = enqueue_stream(s, mode);
        if (st) return st;
    } else {
        SweepArgs h;
        HIP_TRY(put_args(s, mode, 1, &h));
        HIP_TRY(sweep_launch(h, s->dtab + 1, s->plan, s->stream));
    }
    hsp_status st = sync_state(s);
    if (st) return st;
    if (which & HSP_STEP_ADVANCE) {
        // a stepped sweep records no draw: move the draw base with it
        s->sweeps_done += 1;
        s->draw_base += 1;
        Ctrl c;
        HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        c.draw_base = (uint32_t)s->draw_base;
        HIP_TRY(hipMemcpy(s->ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice));
    }
    return HSP_OK;
}

hsp_status hsp_get_debug(hsp_state* s, float* z, int32_t* attempt, double* b) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    if ((z || attempt) && !s->opt.debug_store_z)
        return fail(s, HSP_EINVAL, "create the state with debug_store_z = 1");
    HIP_TRY(hipStreamSynchronize(s->stream));
    const size_t N = s->x.N;
    if (z) HIP_TRY(hipMemcpy(z, s->zdbg, N * sizeof(float), hipMemcpyDeviceToHost));
    if (attempt) HIP_TRY(hipMemcpy(attempt, s->adbg, N * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (b) HIP_TRY(hipMemcpy(b, s->b, s->x.p * sizeof(double), hipMemcpyDeviceToHost));
    return HSP_OK;
}

hsp_status hsp_get_gram(hsp_state* s, double* G) {
    if (!s || !G) return HSP_EINVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(G, s->G, (size_t)s->x.p * s->x.p * sizeof(double), hipMemcpyDeviceToHost));
    return HSP_OK;
}

hsp_status hsp_get_counters(hsp_state* s, uint64_t* clamps, uint32_t* max_attempts) {
    if (!s) return HSP_EINVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    Ctrl c;
    HIP_TRY(hipMemcpy(&c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    if (clamps) *clamps = c.clamps;
    if (max_attempts) *max_attempts = c.max_attempts;
    return HSP_OK;
}

hsp_status hsp_set_timing(hsp_state* s, int32_t enable) {
    if (!s) return HSP_EINVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->timer.reset();
    s->timing = enable != 0;
    return HSP_OK;
}

hsp_status hsp_get_timing(hsp_state* s, double* zpass_ms, double* sweep_ms, int64_t* n) {
    if (!s) return HSP_EINVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    double mean = 0.0, span = 0.0;
    int64_t cnt = 0;
    HIP_TRY(s->timer.result(&mean, &span, &cnt));
    // one kernel per sweep: the z pass and the p-side group share the launch
    if (zpass_ms) *zpass_ms = mean;
    if (sweep_ms) *sweep_ms = span;
    if (n) *n = cnt;
    return HSP_OK;
}

hsp_status hsp_set_phase_trace(hsp_state* s, int32_t enable) {
    if (!s) return HSP_EINVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->sd_mode = 0;  // streamed launch descriptions carry the trace pointer
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    if (s->trace) {
        (void)hipFree(s->trace);
        s->trace = nullptr;
    }
    if (enable) {
        HIP_TRY(dalloc(&s->trace, (size_t)s->plan.capacity * kTraceSlots));
        HIP_TRY(hipMemsetAsync(s->trace, 0, (size_t)s->plan.capacity * kTraceSlots * 8, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    SweepArgs h;
    HIP_TRY(put_args(s, kModeSweep, 0, &h));
    return HSP_OK;
}

hsp_status hsp_get_phase_trace(hsp_state* s, uint64_t* out, int64_t* group_blocks, int64_t* slots,
                               double* ticks_per_us) {
    if (!s) return HSP_EINVAL;
    if (!s->trace) return fail(s, HSP_EINVAL, "enable the trace with hsp_set_phase_trace first");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (out)
        HIP_TRY(hipMemcpy(out, s->trace, (size_t)s->plan.gp * kTraceSlots * 8, hipMemcpyDeviceToHost));
    if (group_blocks) *group_blocks = s->plan.gp;
    if (slots) *slots = kTraceSlots;
    if (ticks_per_us) *ticks_per_us = (double)s->timeout_ticks / 2e6;
    return HSP_OK;
}

namespace {
// Arguments of hsp_gram as a layout of the Gram kernels, or an error text.
const char* gram_args(const void* X, int32_t x_type, int64_t N, int64_t p, int64_t ld, const double* G,
                      XLayout* x) {
    if (!X || !G) return "X and G must not be NULL";
    if (x_type != HSP_X_F32 && x_type != HSP_X_BF16) return "x_type must be HSP_X_F32 or HSP_X_BF16";
    if (N < 1 || p < 1 || ld < p) return "need N >= 1, p >= 1 and ld >= p";
    if (N >= (int64_t(1) << 32) || ld >= (int64_t(1) << 32)) return "N and ld must be below 2^32";
    x->X = dev_ptr(X);
    x->xtype = x_type;
    x->N = (uint32_t)N;
    x->p = (uint32_t)p;
    x->ld = (uint32_t)ld;
    return nullptr;
}

hsp_status gram_device(int* num_cus) {
    hsp_state* s = nullptr;  // HIP_TRY reports through the creation error text
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(num_cus, hipDeviceAttributeMultiprocessorCount, dev));
    return HSP_OK;
}
}  // namespace

hsp_status hsp_gram(const void* X, int32_t x_type, int64_t N, int64_t p, int64_t ld, double* G,
                    void* hip_stream) {
    hsp_state* s = nullptr;
    XLayout x{};
    if (const char* msg = gram_args(X, x_type, N, p, ld, G, &x)) return fail(nullptr, HSP_EINVAL, msg);
    int num_cus = 0;
    if (hsp_status st = gram_device(&num_cus)) return st;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double* work = nullptr;
    HIP_TRY(dalloc(&work, gram_work_doubles(x, num_cus)));
    hipError_t e = gram_launch(x, nullptr, G, work, num_cus, st);
    if (!e) e = hipStreamSynchronize(st);
    (void)hipFree(work);
    HIP_TRY(e);
    return HSP_OK;
}

hsp_status hsp_gram_noalloc(const void* X, int32_t x_type, int64_t N, int64_t p, int64_t ld, double* G,
                            void* hip_stream) {
    hsp_state* s = nullptr;
    XLayout x{};
    if (const char* msg = gram_args(X, x_type, N, p, ld, G, &x)) return fail(nullptr, HSP_EINVAL, msg);
    int num_cus = 0;
    if (hsp_status st = gram_device(&num_cus)) return st;
    const size_t need = gram_pair_doubles(x, num_cus);
    if (need > kGramScratchDoubles)
        return fail(nullptr, HSP_EINVAL,
                    "hsp_gram_noalloc: one tile pair needs " + std::to_string(need * 8) +
                        " bytes of workspace, more than the fixed " + std::to_string(kGramScratchDoubles * 8) +
                        " bytes");
    double* work = nullptr;
    HIP_TRY(gram_scratch(&work));
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(gram_launch_chunked(x, nullptr, G, work, kGramScratchDoubles, num_cus, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HSP_OK;
}

hsp_status hsp_sort_rows(hsp_state* s) {
    if (!s) return HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    if (s->streamed || s->in_batch)
        return fail(s, HSP_EINVAL, "rows can be reordered only for a lone chain with X in device memory");
    const uint32_t N = s->x.N;
    const size_t bytes = (size_t)N * s->x.ld * (s->x.xtype == 0 ? 4 : 2);
    HIP_TRY(hipStreamSynchronize(s->stream));
    // the key of every stored row, ordered on the host (ties keep their order)
    float* key = nullptr;
    HIP_TRY(dalloc(&key, N));
    std::vector<float> kh(N);
    hipError_t e = row_key_launch(s->x, s->beta32, s->y, key, s->stream);
    if (!e) e = hipMemcpyAsync(kh.data(), key, (size_t)N * 4, hipMemcpyDeviceToHost, s->stream);
    if (!e) e = hipStreamSynchronize(s->stream);
    (void)hipFree(key);
    HIP_TRY(e);
    std::vector<uint32_t> perm(N);
    for (uint32_t i = 0; i < N; ++i) perm[i] = i;
    std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) { return kh[a] < kh[b]; });
    uint32_t* dperm = nullptr;
    void* Xo = nullptr;
    uint8_t* yo = nullptr;
    uint32_t* ido = nullptr;
    e = dalloc(&dperm, N);
    if (!e) e = hipMalloc(&Xo, bytes);
    if (!e) e = dalloc(&yo, N);
    if (!e) e = dalloc(&ido, N);
    if (!e) e = hipMemcpyAsync(dperm, perm.data(), (size_t)N * 4, hipMemcpyHostToDevice, s->stream);
    if (!e) e = gather_rows_launch(s->x, dperm, Xo, s->y, yo, s->row_id, ido, s->stream);
    if (!e) e = hipStreamSynchronize(s->stream);
    if (dperm) (void)hipFree(dperm);
    if (e) {
        if (Xo) (void)hipFree(Xo);
        if (yo) (void)hipFree(yo);
        if (ido) (void)hipFree(ido);
        HIP_TRY(e);
    }
    (void)hipFree(s->Xbuf);
    (void)hipFree(s->y);
    if (s->row_id) (void)hipFree(s->row_id);
    s->Xbuf = Xo;
    s->x.X = dev_ptr(static_cast<const void*>(Xo));
    s->y = yo;
    s->row_id = ido;
    SweepArgs h;
    HIP_TRY(put_args(s, kModeSweep, 0, &h));
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    return HSP_OK;
}

hsp_status hsp_get_plan(hsp_state* s, int64_t* group_blocks, int64_t* z_blocks, int64_t* static_pct,
                        int64_t* unit, char* note, int64_t note_cap) {
    if (!s) return HSP_EINVAL;
    if (group_blocks) *group_blocks = s->plan.gp;
    if (z_blocks) *z_blocks = s->plan.gz;
    if (static_pct) *static_pct = s->plan.static_pct;
    if (unit) *unit = s->plan.unit;
    if (note && note_cap > 0) std::snprintf(note, (size_t)note_cap, "%s", s->plan_note.c_str());
    return HSP_OK;
}

hsp_status hsp_batch_get_plan(hsp_batch* b, int64_t* mc_blocks, int64_t* bw_pct, int64_t* packs, char* note,
                              int64_t note_cap) {
    if (!b) return HSP_EINVAL;
    // pack_max is part of the note
    if (mc_blocks) *mc_blocks = b->mc_gz;
    if (bw_pct) *bw_pct = b->bw_pct;
    if (packs) *packs = (int64_t)b->packs.size();
    if (note && note_cap > 0) std::snprintf(note, (size_t)note_cap, "%s", b->plan_note.c_str());
    return HSP_OK;
}

hsp_status hsp_batch_set_shape(hsp_batch* b, int32_t zq_kib, int32_t pre_blocks) {
    if (!b) return HSP_EINVAL;
    if (zq_kib < 0 || zq_kib > 4096) return batch_fail(b, HSP_EINVAL, "zq_kib must lie in [0, 4096]");
    if (pre_blocks < 0 || pre_blocks > 4096) return batch_fail(b, HSP_EINVAL, "pre_blocks must lie in [0, 4096]");
    free_packs(b);  // planned again at the next sweep
    b->zq_kib = (uint32_t)zq_kib;
    b->pre_gp = (uint32_t)pre_blocks;
    b->autotune = false;
    b->plan_note = "zq=" + std::to_string(zq_kib) + " pre=" + std::to_string(pre_blocks) + " (set)";
    return HSP_OK;
}

hsp_status hsp_tune_key(hsp_state* s, char* key, int64_t cap) {
    if (!s || !key || cap < 1) return HSP_EINVAL;
    const std::string k = sweep_tune_key(s);
    if ((int64_t)k.size() >= cap) return fail(s, HSP_EINVAL, "key buffer too small");
    std::memcpy(key, k.c_str(), k.size() + 1);
    return HSP_OK;
}

hsp_status hsp_tune_cache_put(const char* path, const char* key, const char* value) {
    if (!path || !key || !value) return fail(nullptr, HSP_EINVAL, "NULL argument");
    if (!tune_cache_put(path, key, value)) return fail(nullptr, HSP_EINVAL, "cache write failed or bad key/value");
    return HSP_OK;
}

hsp_status hsp_tune_cache_get(const char* path, const char* key, char* value, int64_t cap) {
    if (!path || !key || !value || cap < 1) return fail(nullptr, HSP_EINVAL, "bad arguments");
    std::string v;
    if (!tune_cache_get(path, key, &v)) return fail(nullptr, HSP_ERANGE, "no cache entry");
    if ((int64_t)v.size() >= cap) return fail(nullptr, HSP_EINVAL, "value buffer too small");
    std::memcpy(value, v.c_str(), v.size() + 1);
    return HSP_OK;
}

hsp_status hsp_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out) {
    hsp_state* s = nullptr;
    if (!ctr || !out || n < 0 || n > (int64_t(1) << 28)) return fail(nullptr, HSP_EINVAL, "bad arguments");
    if (n == 0) return HSP_OK;
    uint32_t *dc = nullptr, *dout = nullptr;
    HIP_TRY(dalloc(&dc, 4 * (size_t)n));
    hipError_t e = dalloc(&dout, 4 * (size_t)n);
    if (!e) e = hipMemcpy(dc, ctr, 16 * (size_t)n, hipMemcpyHostToDevice);
    if (!e) e = philox_test_launch(seed, dc, (uint32_t)n, dout, nullptr);
    if (!e) e = hipDeviceSynchronize();
    if (!e) e = hipMemcpy(out, dout, 16 * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(dc);
    if (dout) (void)hipFree(dout);
    HIP_TRY(e);
    return HSP_OK;
}

hsp_status hsp_read_ceiling(hsp_state* s, int32_t iters, double* ms_per_pass, double* bytes_per_pass) {
    if (!s || iters < 1 || !ms_per_pass) return s ? fail(s, HSP_EINVAL, "bad arguments") : HSP_EINVAL;
    if (s->poisoned) return HSP_EPOISONED;
    const size_t esz = s->x.xtype == 0 ? 4 : 2;
    const size_t bytes = (size_t)s->x.N * s->x.ld * esz;
    if (s->streamed) {
        // the link a streamed sweep is bound by: X copied from the pinned
        // host buffer into the device chunk buffers, chunk by chunk
        const size_t row_bytes = (size_t)s->x.ld * esz;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipStreamSynchronize(s->stream));
        HIP_TRY(hipEventCreate(&e0));
        hipError_t e = hipEventCreate(&e1);
        for (int i = -1; !e && i < iters; ++i) {
            if (i == 0) e = hipEventRecord(e0, s->stream);
            for (uint32_t c = 0; !e && c < s->nchunks; ++c) {
                const size_t r0 = (size_t)c * s->chunk_rows;
                const size_t rows = std::min<size_t>(s->chunk_rows, s->x.N - r0);
                e = hipMemcpyAsync(s->stage[c & 1], static_cast<const char*>(s->Xhost) + r0 * row_bytes,
                                   rows * row_bytes, hipMemcpyHostToDevice, s->stream);
            }
        }
        if (!e) e = hipEventRecord(e1, s->stream);
        if (!e) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (!e) e = hipEventElapsedTime(&ms, e0, e1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        HIP_TRY(e);
        *ms_per_pass = ms / iters;
        if (bytes_per_pass) *bytes_per_pass = (double)bytes;
        return HSP_OK;
    }
    float* sink = nullptr;
    HIP_TRY(dalloc(&sink, 1));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (!e) e = hipEventCreate(&e1);
    for (int w = 0; !e && w < 2; ++w) e = stream_read_launch(s->Xbuf, bytes, s->num_cus, sink, s->stream);
    if (!e) e = hipEventRecord(e0, s->stream);
    for (int i = 0; !e && i < iters; ++i) e = stream_read_launch(s->Xbuf, bytes, s->num_cus, sink, s->stream);
    if (!e) e = hipEventRecord(e1, s->stream);
    if (!e) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (!e) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    HIP_TRY(e);
    *ms_per_pass = ms / iters;
    if (bytes_per_pass) *bytes_per_pass = (double)bytes;
    return HSP_OK;
}

hsp_status hsp_tile_schedule(int64_t nt, int64_t gp, int32_t inverse, uint32_t* tasks, int64_t cap,
                             uint32_t* off, int64_t* n_tasks) {
    if (nt < 1 || nt > kMaxP / kTile || gp < 1 || gp > 4096 || inverse < -1 || inverse > 1 || !n_tasks)
        return fail(nullptr, HSP_EINVAL, "bad arguments");
    std::vector<uint32_t> t, o;
    chol_schedule((uint32_t)nt, (uint32_t)gp, &t, &o, inverse < 0 ? with_inverse((uint32_t)nt) : inverse != 0);
    *n_tasks = (int64_t)t.size();
    if ((int64_t)t.size() > cap || !tasks || !off)
        return fail(nullptr, HSP_ERANGE, "task buffer too small");
    std::copy(t.begin(), t.end(), tasks);
    std::copy(o.begin(), o.end(), off);
    return HSP_OK;
}

}  // extern "C"
