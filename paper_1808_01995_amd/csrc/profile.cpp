// Per-kernel device timing with HIP events (enabled on demand), whole runs
// of step launches timed as one span, and per-mode counts of step launches.
#include <atomic>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace wf {

namespace {

constexpr int kKinds = 6;         // WF_KERNEL_STEP .. WF_KERNEL_STEP2_RUN
constexpr int kCounted = kModeCount + 1;   // step modes, then two-update launches

struct Rec {
    int kind;
    hipEvent_t a, b;
    int64_t count;                // launches the record covers
};

std::mutex g_mu;
int g_on = 0;                     // sampling stride, 0 = off
bool g_runs = false;              // whole runs of step launches timed as one span
int64_t g_seen[kKinds] = {};      // launches seen per kind while enabled
std::vector<Rec> g_recs;          // recorded, not yet read
std::vector<hipEvent_t> g_free;   // reusable events
double g_ms[kKinds] = {};
int64_t g_n[kKinds] = {};
std::atomic<int64_t> g_launches[kCounted];   // step launches per mode (always counted)

hipEvent_t get_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    // timing-only events: no system-scope fence (its cache writeback and
    // invalidation would otherwise slow the bracketed kernel)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Fold finished records into the totals (caller holds the lock).
wf_status drain(bool wait) {
    size_t keep = 0;
    for (size_t i = 0; i < g_recs.size(); ++i) {
        Rec& r = g_recs[i];
        if (wait) {
            if (hipEventSynchronize(r.b) != hipSuccess) return fail(WF_E_HIP, "event sync");
        } else if (hipEventQuery(r.b) != hipSuccess) {
            g_recs[keep++] = r;
            continue;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.kind >= 0 && r.kind < kKinds) {
            g_ms[r.kind] += ms;
            g_n[r.kind] += r.count;
        }
        g_free.push_back(r.a);
        g_free.push_back(r.b);
    }
    g_recs.resize(keep);
    (void)hipGetLastError();
    return WF_OK;
}

}  // namespace

bool profiling_active() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on > 0 || g_runs;
}

void count_step_launch(int mode) {
    if (mode >= 0 && mode < kCounted) g_launches[mode].fetch_add(1, std::memory_order_relaxed);
}

RunSpan::RunSpan(hipStream_t st, int k) : s(st), kind(k) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_runs) return;
    if (g_recs.size() > 4096) drain(false);
    a = get_event();
    b = get_event();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) g_free.push_back(a);
        if (b) g_free.push_back(b);
        a = b = nullptr;
    }
}

void RunSpan::finish(int64_t launches) {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (launches > 0 && hipEventRecord(b, s) == hipSuccess) {
        g_recs.push_back({kind, a, b, launches});
    } else {
        g_free.push_back(a);
        g_free.push_back(b);
    }
    a = b = nullptr;
}

RunSpan::~RunSpan() {
    if (!a) return;   // finished, or not timing
    std::lock_guard<std::mutex> lk(g_mu);
    g_free.push_back(a);
    g_free.push_back(b);
}

ProfScope::ProfScope(int k, hipStream_t st) : kind(k), s(st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_on <= 0 || k < 0 || k >= kKinds || k == WF_KERNEL_STEP_RUN || k == WF_KERNEL_STEP2_RUN) return;
    if (g_seen[k]++ % g_on != 0) return;
    if (g_recs.size() > 4096) drain(false);
    a = get_event();
    b = get_event();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) g_free.push_back(a);
        if (b) g_free.push_back(b);
        a = b = nullptr;
    }
}

ProfScope::~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipEventRecord(b, s) == hipSuccess) {
        g_recs.push_back({kind, a, b, 1});
    } else {
        g_free.push_back(a);
        g_free.push_back(b);
    }
}

}  // namespace wf

using namespace wf;

extern "C" {

wf_status wf_profile_enable(int on) {
    if (on < 0) return fail(WF_E_ARG, "negative profiling stride");
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on;
    for (int k = 0; k < kKinds; ++k) g_seen[k] = 0;
    return WF_OK;
}

wf_status wf_profile_runs_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_runs = on != 0;
    return WF_OK;
}

wf_status wf_profile_step_launches(int mode, int64_t* count, int reset) {
    if (mode < 0 || mode >= kCounted) return fail(WF_E_ARG, "unknown step mode %d", mode);
    if (count) *count = g_launches[mode].load();
    if (reset)
        for (int k = 0; k < kCounted; ++k) g_launches[k].store(0);
    return WF_OK;
}

wf_status wf_profile_read(int kind, double* total_ms, int64_t* launches, int reset) {
    if (kind < 0 || kind >= kKinds) return fail(WF_E_ARG, "unknown kernel kind %d", kind);
    std::lock_guard<std::mutex> lk(g_mu);
    wf_status st = drain(true);
    if (st != WF_OK) return st;
    if (total_ms) *total_ms = g_ms[kind];
    if (launches) *launches = g_n[kind];
    if (reset)
        for (int k = 0; k < kKinds; ++k) {
            g_ms[k] = 0.0;
            g_n[k] = 0;
        }
    return WF_OK;
}

}
