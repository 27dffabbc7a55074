// Serving engine: continuous batching of forward and gradient requests on one
// GPU under an HBM budget.
//
// * The budget is one device allocation made at creation, sub-allocated on the
//   host (no hipMalloc/hipFree while serving, so no device-wide syncs).
// * submit() queues a request; admission is FIFO by footprint against the
//   budget and the slot limit, re-run whenever a request completes.
// * Small forward shots (<= kSmallPoints computational nodes: grids whose
//   update moves less data than a kernel launch costs in time) are batched: a
//   batcher thread advances every active small grid together, kBatchSteps
//   time steps per iteration, one k_step_batch launch per step per (dimension,
//   order, tile) group; requests join and leave between iterations, so
//   arrivals are admitted while others are on the GPU and their steps share
//   launches. Two iterations are in flight: arrivals are set up on a second
//   stream and the next iteration is enqueued while the device runs the
//   current one, so the device does not wait for the host between them. The
//   arithmetic of every grid is independent of the batch.
// * Other requests (large grids, gradients) run on worker threads, each with
//   its own non-blocking stream, concurrently with the batch. A free worker
//   takes the admitted request with the earliest expected completion (arrival
//   time plus its estimated run time alone): short requests pass long ones
//   that arrived at about the same time, and a long request is passed only
//   by requests that would finish before it anyway. At most one heavy
//   request (a grid above kSmallPoints nodes) runs at a time: one such grid
//   already fills the GPU at its HBM roofline, and two side by side share
//   the bandwidth while evicting each other from the Infinity Cache (two
//   concurrent 3D shots took 7 % longer than the same shots in turn).
#include <algorithm>
#include <climits>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <new>
#include <thread>
#include <vector>

#include "runtime.h"

namespace wf {

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------
struct Arena {
    char* base = nullptr;
    int64_t size = 0;
    int64_t used = 0;
    std::mutex mu;
    std::map<int64_t, int64_t> free_;   // offset -> size
    std::map<int64_t, int64_t> live;    // offset -> size
};

Arena* arena_create(int64_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(WF_E_NOMEM, "cannot allocate a %lld-byte device arena", (long long)bytes);
        return nullptr;
    }
    Arena* a = new (std::nothrow) Arena();
    if (!a) {
        hipFree(p);
        fail(WF_E_NOMEM, "host allocation");
        return nullptr;
    }
    a->base = static_cast<char*>(p);
    a->size = bytes;
    a->free_[0] = bytes;
    return a;
}

void arena_destroy(Arena* a) {
    if (!a) return;
    hipFree(a->base);
    delete a;
}

void* arena_alloc(Arena* a, int64_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    std::lock_guard<std::mutex> lk(a->mu);
    for (auto it = a->free_.begin(); it != a->free_.end(); ++it) {
        if (it->second >= bytes) {
            const int64_t off = it->first, sz = it->second;
            a->free_.erase(it);
            if (sz > bytes) a->free_[off + bytes] = sz - bytes;
            a->live[off] = bytes;
            a->used += bytes;
            return a->base + off;
        }
    }
    return nullptr;
}

void arena_free(Arena* a, void* p) {
    std::lock_guard<std::mutex> lk(a->mu);
    const int64_t off = static_cast<char*>(p) - a->base;
    auto it = a->live.find(off);
    if (it == a->live.end()) return;
    int64_t start = off, sz = it->second;
    a->used -= sz;
    a->live.erase(it);
    auto nx = a->free_.lower_bound(start);
    if (nx != a->free_.end() && nx->first == start + sz) {
        sz += nx->second;
        nx = a->free_.erase(nx);
    }
    if (nx != a->free_.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == start) {
            start = pv->first;
            sz += pv->second;
            a->free_.erase(pv);
        }
    }
    a->free_[start] = sz;
}

int64_t arena_used(const Arena* a) { return a ? a->used : 0; }

int64_t arena_largest_free(Arena* a) {
    std::lock_guard<std::mutex> lk(a->mu);
    int64_t m = 0;
    for (auto& kv : a->free_) m = std::max(m, kv.second);
    return m;
}

}  // namespace wf

using namespace wf;

namespace {

// batched if the grid has at most this many nodes (every 2D grid up to
// 2128^2; 3D grids of 9 M+ nodes ran 6 % slower batched than alone, their
// fields no longer sharing the Infinity Cache with nobody)
constexpr int64_t kSmallPoints = (int64_t)5 << 20;
constexpr int kBatchSteps = 32;                        // steps per batch iteration
constexpr int kWorkers = 2;                            // threads for large requests and gradients
constexpr int kGradShare = 2 * kWorkers;               // a gradient's checkpoints take <= budget / kGradShare
constexpr int kThrottleSteps = 16;                     // step launches a worker keeps queued (x2)

struct EJob {
    uint64_t ticket = 0;
    wf_request rq{};
    std::vector<double> src, rec;
    bool small = false;
    bool tiny = false;      // forward shot whose two fields fit one work-group's LDS (resident team)
    int path = 2;           // where it ran: 0 resident team, 1 batched launches, 2 a worker
    bool heavy = false;     // grid above kSmallPoints nodes: runs alone among the workers' jobs
    bool counted = false;   // counted in heavy_running while it runs
    double due = 0.0;       // arrival (s, steady clock) + estimated run time alone
    int64_t foot = 0;       // bytes reserved at admission
    int64_t grad_cap = 0;   // bytes the gradient's checkpoints may use
    wf_status st = WF_OK;
    Model* md = nullptr;
    BatchFwd bf;
    const PointSet* ps_src = nullptr;
    const PointSet* ps_rec = nullptr;
    DevBuf inc;                   // resident team: the source increments of every step
    hipEvent_t ready = nullptr;   // recorded on the submitter's stream: the inputs are complete
    ~EJob() {
        if (ready) (void)hipEventDestroy(ready);
    }
    // make work on `s` wait until the submitter's inputs are complete
    wf_status wait_inputs(hipStream_t s) const {
        return ready ? hip_check(hipStreamWaitEvent(s, ready, 0), "wait for the request's inputs") : WF_OK;
    }
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// run time of a request alone, from its streamed bytes at ~5 TB/s: 16 B per
// node per update for a forward shot; a gradient adds the residual forward
// sweep, recomputation and the 28-byte imaging sweep (about 3 forward shots)
double estimate_seconds(const wf_request* r, int64_t npoints) {
    const double fwd = 16.0 * (double)npoints * (double)std::max(r->nt - 1, 0) / 5e12;
    return r->kind == WF_REQ_GRADIENT ? 3.0 * fwd : fwd;
}

int64_t field_bytes_of(const wf_geom* g) {
    Layout L;
    L.init(g);
    return L.field_bytes();
}

// Increment slots of the fused injection of a point set, bounded from above
// without building its tables: an entry is one (x, y, z / 4) group of nodes
// (the 4 z nodes of the owning thread; z tiles start at multiples of 4), with
// 4 slots, and every corner node of every point's cell may be one.
int64_t fused_slots_bound(const wf_geom* g, const Layout& L, int npts, const double* xyz) {
    const int D = g->ndim;
    const int64_t n[3] = {L.nx, D == 3 ? L.ny : 1, L.nz};
    std::vector<int64_t> keys;
    keys.reserve((size_t)npts << D);
    for (int p = 0; p < npts; ++p) {
        int64_t base[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            const int la = D == 3 ? a : (a == 0 ? 0 : 2);   // layout axis of coordinate a
            const double s = (xyz[(size_t)p * D + a] - g->origin[a]) / g->h[a] + g->nbl;
            int64_t i = std::isfinite(s) ? (int64_t)std::floor(s) : 0;
            base[la] = std::max<int64_t>(0, std::min<int64_t>(i, n[la] - 2));
        }
        for (int c = 0; c < (1 << D); ++c) {
            int64_t v[3] = {base[0], base[1], base[2]};
            v[0] += c & 1;
            if (D == 3) v[1] += (c >> 1) & 1;
            v[2] += (c >> (D - 1)) & 1;
            keys.push_back((v[0] * n[1] + v[1]) * ((n[2] + 3) / 4) + v[2] / 4);
        }
    }
    std::sort(keys.begin(), keys.end());
    const int64_t entries = std::unique(keys.begin(), keys.end()) - keys.begin();
    return 4 * entries;
}

}  // namespace

struct wf_engine {
    Arena* arena = nullptr;
    int64_t budget = 0;
    int max_slots = 1;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<EJob*> pending;
    std::deque<EJob*> small_ready;
    std::deque<EJob*> large_ready;
    std::deque<EJob*> tiny_ready;
    bool teams_on = true;       // tiny forward shots go to resident teams
    std::deque<std::pair<uint64_t, wf_status>> done;
    int64_t reserved = 0;
    int running = 0;
    int64_t served[3] = {0, 0, 0};   // completed requests by path: resident teams, batched launches, workers
    int heavy_running = 0;      // heavy requests on the workers (0 or 1)
    int64_t completed = 0;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::vector<std::thread> threads;

    // FIFO admission (caller holds mu)
    void admit() {
        while (!pending.empty() && running < max_slots && reserved + pending.front()->foot <= budget) {
            EJob* j = pending.front();
            pending.pop_front();
            reserved += j->foot;
            ++running;
            if (j->tiny && teams_on) {
                j->path = 0;
                tiny_ready.push_back(j);
            } else if (j->small) {
                j->path = 1;
                small_ready.push_back(j);
            } else {
                j->path = 2;
                large_ready.push_back(j);
            }
        }
        cv_work.notify_all();
    }

    void complete(EJob* j) {
        std::lock_guard<std::mutex> lk(mu);
        ++served[j->path];
        if (j->counted) --heavy_running;
        reserved -= j->foot;
        --running;
        ++completed;
        done.emplace_back(j->ticket, j->st);
        delete j;
        admit();
        cv_done.notify_all();
    }

    void run_large(EJob* j, hipStream_t s);
    void worker();
    void batcher();
    void teams();
};

// footprint estimate of a request (bytes of the arena it may occupy); the
// coordinates are the host copies held by the job
static wf_status footprint(const wf_request* r, const double* src_xyz, const double* rec_xyz,
                           int64_t budget, EJob* j) {
    Layout L;
    L.init(&r->geom);
    const int64_t fb = L.field_bytes();
    const int64_t dense = L.npoints * 4;
    const int K = 1 << r->geom.ndim;
    const int64_t pts = (int64_t)(r->nsrc + r->nrec) * K;
    const int64_t tables = pts * 64 + (int64_t)L.nx * 4 * 1024 + ((int64_t)16 << 20);
    // precomputed increments of the fused injection: one float per slot and row
    const int64_t inc_src = (int64_t)r->nt * fused_slots_bound(&r->geom, L, r->nsrc, src_xyz) * 4;
    const int64_t inc_rec = (int64_t)r->nt * fused_slots_bound(&r->geom, L, r->nrec, rec_xyz) * 4;
    const int64_t model = dense + 3 * fb + ((int64_t)1 << 20);
    if (r->kind == WF_REQ_FORWARD) {
        j->foot = model + inc_src + tables;
        j->small = L.npoints <= kSmallPoints;
        j->heavy = !j->small;
        j->tiny = team_fits(L.nx, L.ny, L.nz);
    } else {
        // record scratch (predicted data, residual, partial sums), both
        // increment tables, adjoint pair and gradient, and a checkpoint pool:
        // every forward field if they fit in the gradient's share of the
        // budget (the workers' gradients together hold at most half of it),
        // else a revolve pool of that size (the arena is allocated once, so
        // a larger pool costs no allocation, only fewer recomputed steps)
        const int64_t l = r->nt - 1;
        const int64_t rec_bytes = 2 * (int64_t)r->nt * r->nrec * 4 + ((int64_t)1 << 20);
        const int64_t fixed = model + inc_src + inc_rec + rec_bytes + 3 * fb + tables;
        int64_t pool = std::min<int64_t>((l + 1) * fb, std::max<int64_t>(5 * fb, budget / kGradShare));
        if (fixed + pool > budget) pool = 5 * fb;   // one snapshot, the minimum
        j->grad_cap = 3 * fb + pool + rec_bytes + ((int64_t)1 << 20);
        j->foot = fixed + pool;
        j->small = false;
        j->heavy = L.npoints > kSmallPoints;
    }
    j->due = now_s() + estimate_seconds(r, L.npoints);
    if (j->foot > budget)
        return fail(WF_E_BUDGET, "request needs about %lld bytes, the engine budget is %lld",
                    (long long)j->foot, (long long)budget);
    return WF_OK;
}

void wf_engine::run_large(EJob* j, hipStream_t s) {
    const wf_request& r = j->rq;
    std::unique_ptr<Model> md(new (std::nothrow) Model());
    wf_status st = md ? j->wait_inputs(s) : fail(WF_E_NOMEM, "host allocation");
    if (st == WF_OK) st = md->init(&r.geom, r.m_dev, s);
    const PointSet *src = nullptr, *rec = nullptr;
    if (st == WF_OK) st = md->check_dt(r.dt);
    if (st == WF_OK) st = md->points(r.nsrc, j->src.data(), &src);
    if (st == WF_OK) st = md->points(r.nrec, j->rec.data(), &rec);
    if (st == WF_OK && r.kind == WF_REQ_FORWARD) {
        st = run_forward(*md, r.dt, r.nt, *src, r.src_wav, *rec, r.rec_out, nullptr, 1, s);
        if (st == WF_OK) st = hip_check(hipStreamSynchronize(s), "sync");
    } else if (st == WF_OK) {
        // two wave solves: the residual comes from the gradient's own forward sweep
        double phi = 0.0;
        st = run_gradient(*md, r.dt, r.nt, *src, r.src_wav, *rec, nullptr, r.grad_out, 0, j->grad_cap, s,
                          r.d_obs, r.rec_out, &phi);
        if (st == WF_OK && r.misfit_out) *r.misfit_out = phi;
        if (st == WF_OK) st = hip_check(hipStreamSynchronize(s), "sync");
    }
    md.reset();   // waits for the model's stream
    j->st = st;
}

void wf_engine::worker() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    set_thread_arena(arena, s);
    // a heavy request keeps only a few milliseconds of launches queued, so
    // that requests arriving meanwhile (the batcher's launches, the other
    // worker's) are not queued behind its whole time loop when their streams
    // share a hardware queue
    set_thread_throttle(kThrottleSteps);
    for (;;) {
        EJob* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            // earliest expected completion among the requests this worker may
            // start (no second heavy one while one runs)
            auto pick = [&]() {
                auto best = large_ready.end();
                for (auto it = large_ready.begin(); it != large_ready.end(); ++it) {
                    if ((*it)->heavy && heavy_running > 0) continue;
                    if (best == large_ready.end() || (*it)->due < (*best)->due) best = it;
                }
                return best;
            };
            cv_work.wait(lk, [&] { return (stop && large_ready.empty()) || pick() != large_ready.end(); });
            auto best = pick();
            if (best == large_ready.end()) break;   // stop requested and nothing left
            j = *best;
            large_ready.erase(best);
            if (j->heavy) {
                ++heavy_running;
                j->counted = true;
            }
        }
        try {
            run_large(j, s);
        } catch (...) {
            // a host allocation failed: the request fails (complete() frees
            // its slot and its place as the running heavy request)
            j->st = fail(WF_E_NOMEM, "host allocation failed while serving a request");
        }
        complete(j);
    }
    (void)hipStreamDestroy(s);
    set_thread_arena(nullptr);
}

void wf_engine::batcher() {
    (void)hipSetDevice(device);
    // launches of the batched steps go to `s`; newly admitted grids are set
    // up on `s_setup` meanwhile, and the launches that first include them
    // wait for that set-up on the device
    hipStream_t s = nullptr, s_setup = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    (void)hipStreamCreateWithFlags(&s_setup, hipStreamNonBlocking);
    hipEvent_t setup_ev = nullptr;
    (void)hipEventCreateWithFlags(&setup_ev, hipEventDisableTiming);
    // grids are retired only after the iteration that last used them has run
    // (an event), so freeing their buffers waits for the set-up stream alone
    set_thread_arena(arena, s_setup);
    // Two iterations in flight: while the device runs one, the host sets up
    // arrivals and enqueues the next; each has its own job tables and an
    // event, and the grids that finished in it are completed when its event
    // has fired.
    struct Slot {
        BatchJob* host = nullptr;
        int cap = 0;
        DevBuf dev;
        hipEvent_t ev = nullptr;
        bool armed = false;
        std::vector<EJob*> retiring;
    };
    Slot slot[2];
    for (Slot& sl : slot) (void)hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    int cur = 0;
    auto drain = [&](Slot& sl) {
        if (!sl.armed) return;
        const wf_status st = hip_check(hipEventSynchronize(sl.ev), "batched iteration");
        sl.armed = false;
        std::vector<EJob*> done_jobs;
        done_jobs.swap(sl.retiring);
        for (EJob* j : done_jobs) {
            if (st != WF_OK && j->st == WF_OK) j->st = st;
            delete j->md;
            j->md = nullptr;
            complete(j);
        }
    };
    std::vector<EJob*> active;
    for (;;) {
        std::vector<EJob*> fresh;
        if (active.empty()) {
            drain(slot[0]);
            drain(slot[1]);
        }
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty())
                cv_work.wait(lk, [&] { return stop || !small_ready.empty(); });
            while (!small_ready.empty()) {
                fresh.push_back(small_ready.front());
                small_ready.pop_front();
            }
            if (active.empty() && fresh.empty() && stop) break;
        }
        size_t fresh_in_active = 0;   // fresh grids already moved to `active`
        try {
        // set up newly admitted grids on the set-up stream (their first step
        // joins this iteration)
        for (EJob* j : fresh) {
            const wf_request& r = j->rq;
            j->md = new (std::nothrow) Model();
            wf_status st = j->md ? j->wait_inputs(s_setup) : fail(WF_E_NOMEM, "host allocation");
            if (st == WF_OK) st = j->md->init(&r.geom, r.m_dev, s_setup);
            if (st == WF_OK) st = j->md->check_dt(r.dt);
            if (st == WF_OK) st = j->md->points(r.nsrc, j->src.data(), &j->ps_src);
            if (st == WF_OK) st = j->md->points(r.nrec, j->rec.data(), &j->ps_rec);
            if (st == WF_OK)
                st = batch_forward_begin(*j->md, r.dt, r.nt, *j->ps_src, r.src_wav, *j->ps_rec, r.rec_out, s_setup,
                                         j->bf);
            if (st == WF_E_STATE) {
                // not batchable (too many sources in one block): run it alone
                st = run_forward(*j->md, r.dt, r.nt, *j->ps_src, r.src_wav, *j->ps_rec, r.rec_out, nullptr, 1,
                                 s_setup);
                if (st == WF_OK) st = hip_check(hipStreamSynchronize(s_setup), "sync");
                j->bf.n = r.nt - 1;
                j->bf.nt = r.nt;
                j->bf.rec = nullptr;
            }
            j->st = st;
            active.push_back(j);
            ++fresh_in_active;
        }
        if (!fresh.empty()) {
            wf_status st = hip_check(hipEventRecord(setup_ev, s_setup), "event");
            if (st == WF_OK) st = hip_check(hipStreamWaitEvent(s, setup_ev, 0), "wait for set-up");
            if (st != WF_OK)
                for (EJob* j : fresh) j->st = st;
        }
        // one iteration: kBatchSteps steps of every active grid, one launch
        // per step per (dimension, order, tile) group
        std::map<std::tuple<int, int, int>, std::vector<EJob*>> groups;
        for (EJob* j : active)
            if (j->st == WF_OK && j->bf.n < j->bf.nt - 1)
                groups[std::make_tuple(j->md->geom.ndim, j->md->half, j->bf.p.tile)].push_back(j);
        int ntab = 0;
        for (auto& g : groups) ntab += (int)g.second.size();
        Slot& sl = slot[cur];
        drain(sl);   // its tables and its finished grids are free now
        wf_status st = WF_OK;
        if (ntab > 0) {
            if (ntab > sl.cap) {
                if (sl.host) (void)hipHostFree(sl.host);
                sl.host = nullptr;
                sl.cap = 0;
                const int cap = std::max(ntab, 64);
                if (hipHostMalloc(reinterpret_cast<void**>(&sl.host), sizeof(BatchJob) * cap) != hipSuccess) {
                    sl.host = nullptr;
                    st = fail(WF_E_NOMEM, "pinned host table");
                } else {
                    sl.cap = cap;
                    st = sl.dev.alloc((int64_t)sizeof(BatchJob) * cap);
                }
            }
            struct G { int off, n, total, ndim, half, tile; };
            std::vector<G> gl;
            int off = 0;
            for (auto& g : groups) {
                if (st != WF_OK) break;   // no table to fill
                int begin = 0;
                for (size_t q = 0; q < g.second.size(); ++q) {
                    sl.host[off + (int)q] = batch_forward_job(g.second[q]->bf, kBatchSteps, begin);
                    begin += g.second[q]->bf.nblk;
                }
                gl.push_back({off, (int)g.second.size(), begin, std::get<0>(g.first), std::get<1>(g.first),
                              std::get<2>(g.first)});
                off += (int)g.second.size();
            }
            if (st == WF_OK)
                st = hip_check(hipMemcpyAsync(sl.dev.ptr, sl.host, sizeof(BatchJob) * ntab, hipMemcpyHostToDevice, s),
                               "batch table");
            for (int k = 0; k < kBatchSteps && st == WF_OK; ++k)
                for (const G& g : gl)
                    st = hip_check(launch_step_batch(sl.dev.as<BatchJob>() + g.off, g.n, g.total, g.ndim, g.half,
                                                     g.tile, k, s), "batched step");
            for (auto& g : groups)
                for (EJob* j : g.second) {
                    const int steps = std::max(0, std::min(kBatchSteps, j->bf.nt - 1 - j->bf.n));
                    batch_forward_advance(j->bf, steps);
                    if (st != WF_OK) j->st = st;
                }
        }
        // grids done after this iteration: their last record row, then they
        // retire with the iteration's event
        std::vector<EJob*> keep;
        keep.reserve(active.size());   // no allocation once grids start to retire
        for (EJob*& j : active) {
            if (j->st == WF_OK && j->bf.n < j->bf.nt - 1) {
                keep.push_back(j);
                continue;
            }
            if (j->st == WF_OK && j->bf.rec) j->st = batch_forward_finish(j->bf, s);
            sl.retiring.push_back(j);
            j = nullptr;   // handed to the slot: the error path below must not touch it
        }
        active.swap(keep);
        const wf_status se = hip_check(hipEventRecord(sl.ev, s), "event");
        if (se == WF_OK) {
            sl.armed = true;
        } else {
            // no event: wait for the stream instead and retire at once
            (void)hipStreamSynchronize(s);
            for (EJob* j : sl.retiring) j->st = se;
            std::vector<EJob*> done_jobs;
            done_jobs.swap(sl.retiring);
            for (EJob* j : done_jobs) {
                delete j->md;
                j->md = nullptr;
                complete(j);
            }
        }
        cur ^= 1;
        } catch (...) {
            // a host allocation failed: every grid in the batch fails (after
            // the launches already issued have finished), the slots are freed
            (void)hipStreamSynchronize(s);
            (void)hipStreamSynchronize(s_setup);
            for (size_t i = fresh_in_active; i < fresh.size(); ++i) active.push_back(fresh[i]);
            for (Slot& q : slot) {
                for (EJob* j : q.retiring) active.push_back(j);
                q.retiring.clear();
                q.armed = false;
            }
            for (EJob* j : active) {
                if (!j) continue;   // already handed over
                delete j->md;
                j->md = nullptr;
                j->st = fail(WF_E_NOMEM, "host allocation failed while batching");
                complete(j);
            }
            active.clear();
        }
    }
    drain(slot[0]);
    drain(slot[1]);
    for (Slot& sl : slot) {
        if (sl.host) (void)hipHostFree(sl.host);
        sl.dev.reset();
        (void)hipEventDestroy(sl.ev);
    }
    (void)hipEventDestroy(setup_ev);
    (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(s_setup);
    set_thread_arena(nullptr);
}

// Resident teams (k_team): tiny forward shots are set up (model, point
// tables, coefficients) on the thread's own stream and then launched in
// groups of one (dimension, order); a launch's work-groups take its shots in
// turn, each holding its shot's two fields in LDS to the end. Up to
// kTeamLaunches launches run at once, each on its own stream, so shots that
// arrive while others run start at once in the next free one. A launch
// depends on nothing but its table: it never waits for other work.
struct TeamLaunch {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;      // recorded after the launch
    TeamJob* host = nullptr;      // pinned: the table, then the error flag read back after the launch
    int cap = 0;
    DevBuf dev;                   // the table, the shot counter and error flag, barrier counters, exchange
    std::vector<EJob*> jobs;      // in flight
    bool split = false;           // its shots are split over teams of work-groups
    unsigned int* err_host() const { return reinterpret_cast<unsigned int*>(host + cap); }
};

namespace {

constexpr int kTeamLaunches = 4;
constexpr unsigned long long kTeamWaitTicks = 100000000ull;   // 1 s at 100 MHz: a barrier wait that long fails
constexpr int kTeamMaxWidth = 8;
constexpr int kTeamMaxPeriod = 8;

// Work-groups per shot and updates between exchanges. A launch of few shots
// splits each over up to kTeamMaxWidth work-groups (at most one per CU in
// all), each owning at least max(8, M) planes; the period is as long as
// every part's planes allow (period M <= planes owned), up to
// kTeamMaxPeriod. WAVEFD_TEAM_WIDTH (1, 2, 4, 8) and WAVEFD_TEAM_PERIOD
// override within those limits.
void team_split(int n, int min_nx, int half, int cus, int* width, int* period) {
    int w = 1;
    while (w < kTeamMaxWidth && (int64_t)2 * w * n <= cus) w *= 2;
    if (const char* e = std::getenv("WAVEFD_TEAM_WIDTH")) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8) w = v;
    }
    while (w > 1 && min_nx / w < std::max(half, 8)) w /= 2;
    int k = w > 1 ? std::min(kTeamMaxPeriod, (min_nx / w) / half) : 1;
    if (const char* e = std::getenv("WAVEFD_TEAM_PERIOD")) {
        const int v = std::atoi(e);
        if (v >= 1) k = std::min(k, v);
    }
    *width = w;
    *period = std::max(1, k);
}
constexpr int64_t kTeamStagingBytes = (int64_t)8 << 20;   // pinned staging of the set-up uploads of a batch

TeamJob team_job(const Model& md, const PointSet& src, const PointSet& rec, const wf_request& r,
                 const float* inc) {
    TeamJob J;
    std::memset(&J, 0, sizeof J);
    StepParams p;
    md.fill_step(p, r.dt);
    J.ndim = md.geom.ndim;
    J.half = md.half;
    J.nx = md.L.nx;
    J.ny = md.L.ny;
    J.nz = md.L.nz;
    J.nt = r.nt;
    J.nrec = rec.npts;
    J.nnodes = src.nnodes;
    J.c0 = p.c0;
    J.inv2dt = p.inv2dt;
    for (int j = 0; j <= kMaxHalf; ++j) {
        J.wx[j] = p.wx[j];
        J.wy[j] = p.wy[j];
        J.wz[j] = p.wz[j];
    }
    J.sx = md.L.sx;
    J.sy = md.L.sy;
    J.kap = md.kap();
    J.etax = p.etax;
    J.etay = p.etay;
    J.etaz = p.etaz;
    J.noff = src.d_noff.as<int64_t>();
    J.inc = inc;
    J.smp_off = rec.d_off.as<int64_t>();
    J.smp_w = rec.d_w.f();
    J.rec = r.rec_out;
    return J;
}

// the source increments of every step of a resident-team shot, by the
// increment kernel of the other paths over the point set's node tables
wf_status team_increments(const Model& md, const PointSet& src, const wf_request& r, DevBuf& buf,
                          hipStream_t s) {
    if (src.nnodes == 0 || r.nt < 2) return WF_OK;
    const wf_status st = buf.alloc((int64_t)(r.nt - 1) * src.nnodes * 4);
    if (st != WF_OK) return st;
    StepParams p;
    md.fill_step(p, r.dt);
    IncParams ip{};
    ip.inc = buf.f();
    ip.kap = md.kap();
    ip.off = src.d_noff.as<int64_t>();
    ip.eta = src.d_neta.f();
    ip.seg = src.d_seg.as<int>();
    ip.pt = src.d_ept.as<int>();
    ip.w = src.d_ew.f();
    ip.vals = r.src_wav;
    ip.nnodes = src.nnodes;
    ip.npts = src.npts;
    ip.nrows = r.nt - 1;
    ip.inv2dt = p.inv2dt;
    return hip_check(launch_increments(ip, s), "increments");
}

// table of `jobs` into `L` (growing it), then the launch, the read-back of
// its error flag and its event
wf_status team_launch(TeamLaunch& L, const std::vector<EJob*>& jobs, int ndim, int half, int cus,
                      bool split_ok) {
    const int n = (int)jobs.size();
    int min_nx = INT_MAX;
    int64_t max_plane = 0;   // float4 per x plane
    for (const EJob* j : jobs) {
        min_nx = std::min(min_nx, j->md->L.nx);
        max_plane = std::max<int64_t>(max_plane, (int64_t)j->md->L.ny * ((j->md->L.nz + 3) / 4));
    }
    int width = 1, period = 1;
    if (split_ok) team_split(n, min_nx, half, cus, &width, &period);
    L.split = width > 1;
    const int64_t stride = width > 1 ? (int64_t)2 * width * 2 * 2 * period * half * max_plane : 0;   // float4
    const int64_t off_ctl = (int64_t)sizeof(TeamJob) * std::max(n, 256);
    const int64_t off_cnt = off_ctl + 256;
    const int64_t off_exch = (off_cnt + (int64_t)n * 128 + 255) / 256 * 256;
    const int64_t need = off_exch + stride * 16 * n;
    if (n > L.cap) {
        if (L.host) (void)hipHostFree(L.host);
        L.host = nullptr;
        L.cap = 0;
        const int cap = std::max(n, 256);
        if (hipHostMalloc(reinterpret_cast<void**>(&L.host), sizeof(TeamJob) * cap + 256) != hipSuccess) {
            L.host = nullptr;
            return fail(WF_E_NOMEM, "pinned team table");
        }
        L.cap = cap;
    }
    if (L.dev.bytes < need) {
        const wf_status st = L.dev.alloc(need);
        if (st != WF_OK) return st;
    }
    for (int i = 0; i < n; ++i) {
        const EJob& j = *jobs[(size_t)i];
        L.host[i] = team_job(*j.md, *j.ps_src, *j.ps_rec, j.rq, j.inc.f());
    }
    char* base = L.dev.as<char>();
    TeamArgs a;
    a.jobs = reinterpret_cast<const TeamJob*>(base);
    a.next = reinterpret_cast<unsigned int*>(base + off_ctl);
    a.err = a.next + 1;
    a.njobs = n;
    a.width = width;
    a.period = period;
    a.cnt = reinterpret_cast<unsigned int*>(base + off_cnt);
    a.exch = reinterpret_cast<float4*>(base + off_exch);
    a.exch_stride = stride;
    a.limit = kTeamWaitTicks;
    *L.err_host() = 0;
    const int nteams = width > 1 ? std::min(n, std::max(1, cus / width)) : std::min(n, cus);
    wf_status st = hip_check(hipMemcpyAsync(L.dev.ptr, L.host, sizeof(TeamJob) * n, hipMemcpyHostToDevice, L.s),
                             "team table");
    // shot counter, error flag and barrier counters start at zero
    if (st == WF_OK)
        st = hip_check(launch_fill(reinterpret_cast<float*>(a.next), (off_exch - off_ctl) / 4, 0.0f, L.s),
                       "team counters");
    if (st == WF_OK) st = hip_check(launch_team(a, ndim, half, nteams * width, L.s), "team launch");
    if (st == WF_OK)
        st = hip_check(hipMemcpyAsync(L.err_host(), a.err, sizeof(unsigned int), hipMemcpyDeviceToHost, L.s),
                       "team error flag");
    if (st == WF_OK) st = hip_check(hipEventRecord(L.ev, L.s), "event");
    return st;
}

}  // namespace

void wf_engine::teams() {
    (void)hipSetDevice(device);
    hipStream_t s_setup = nullptr;
    wf_status broken = hip_check(hipStreamCreateWithFlags(&s_setup, hipStreamNonBlocking), "stream");
    set_thread_arena(arena, s_setup);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    TeamLaunch launches[kTeamLaunches];
    for (TeamLaunch& L : launches) {
        if (broken == WF_OK) broken = hip_check(hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking), "stream");
        if (broken == WF_OK) broken = hip_check(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming), "event");
    }
    auto finish = [&](EJob* j, wf_status st) {
        if (j->st == WF_OK) j->st = st;
        j->inc.reset();
        delete j->md;
        j->md = nullptr;
        complete(j);
    };
    // set-up of a batch of arrivals is queued without a host wait: small
    // uploads go through pinned staging, the check of each m lands in a
    // pinned slot, and one synchronisation covers the batch
    PinnedStaging staging;
    staging.stream = s_setup;
    if (hipHostMalloc(reinterpret_cast<void**>(&staging.base), kTeamStagingBytes) == hipSuccess)
        staging.size = kTeamStagingBytes;
    else
        staging.base = nullptr;
    unsigned int* host3 = nullptr;   // pinned, 4 per arrival of a batch
    size_t host3_cap = 0;
    std::vector<EJob*> backlog;   // set up, waiting for a free launch
    std::vector<EJob*> pend;      // set up, the check of m pending
    for (;;) {
        bool busy = false;
        for (TeamLaunch& L : launches) busy = busy || !L.jobs.empty();
        std::vector<EJob*> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!busy && backlog.empty()) cv_work.wait(lk, [&] { return stop || !tiny_ready.empty(); });
            else if (tiny_ready.empty()) cv_work.wait_for(lk, std::chrono::microseconds(50));
            while (!tiny_ready.empty()) {
                fresh.push_back(tiny_ready.front());
                tiny_ready.pop_front();
            }
            if (!busy && fresh.empty() && backlog.empty() && stop) break;
        }
        size_t k = 0;   // fresh[k..] not set up yet
        try {
            // set the arrivals up (waiting for their inputs on the set-up
            // stream), then wait once for all of them and check each m and dt
            if (fresh.size() > host3_cap) {
                if (host3) (void)hipHostFree(host3);
                host3 = nullptr;
                host3_cap = 0;
                const size_t cap = std::max<size_t>(fresh.size(), 256);
                if (hipHostMalloc(reinterpret_cast<void**>(&host3), cap * 4 * sizeof(unsigned int)) != hipSuccess)
                    host3 = nullptr;
                else
                    host3_cap = cap;
            }
            if (staging.used > 0) (void)hipStreamSynchronize(s_setup);   // its copies have passed
            staging.used = 0;
            set_thread_staging(staging.base ? &staging : nullptr);
            for (; k < fresh.size(); ++k) {
                EJob* j = fresh[k];
                const wf_request& r = j->rq;
                wf_status st = host3 ? broken : fail(WF_E_NOMEM, "pinned host slots");
                if (st == WF_OK) {
                    j->md = new Model();
                    st = j->wait_inputs(s_setup);
                }
                if (st == WF_OK) st = j->md->init_pending(&r.geom, r.m_dev, s_setup, host3 + 4 * pend.size());
                if (st == WF_OK) st = j->md->points(r.nsrc, j->src.data(), &j->ps_src);
                if (st == WF_OK) st = j->md->points(r.nrec, j->rec.data(), &j->ps_rec);
                if (st == WF_OK) st = j->md->ensure_kap(r.dt, s_setup);
                if (st == WF_OK) st = team_increments(*j->md, *j->ps_src, r, j->inc, s_setup);
                if (st == WF_OK) pend.push_back(j);
                else finish(j, st);
            }
            set_thread_staging(nullptr);
            if (!pend.empty()) {
                const wf_status st = hip_check(hipStreamSynchronize(s_setup), "set-up");
                for (size_t i = 0; i < pend.size(); ++i) {
                    EJob* j = pend[i];
                    wf_status sj = st;
                    if (sj == WF_OK) sj = j->md->finish_m(host3 + 4 * i);
                    if (sj == WF_OK) sj = j->md->check_dt(j->rq.dt);
                    if (sj == WF_OK) backlog.push_back(j);
                    else finish(j, sj);
                }
                pend.clear();
            }
            // retire finished launches
            for (TeamLaunch& L : launches) {
                if (L.jobs.empty()) continue;
                const hipError_t q = hipEventQuery(L.ev);
                if (q == hipErrorNotReady) continue;
                wf_status st = q == hipSuccess ? WF_OK : hip_check(q, "team launch");
                if (st == WF_OK && *L.err_host() != 0)
                    st = fail(WF_E_STATE, "a resident team's barrier wait timed out");
                std::vector<EJob*> done_jobs;
                done_jobs.swap(L.jobs);
                for (EJob* j : done_jobs) finish(j, st);
            }
            // launch what waits, one (ndim, half) group per free launch
            while (!backlog.empty()) {
                TeamLaunch* L = nullptr;
                for (TeamLaunch& c : launches)
                    if (c.jobs.empty() && !L) L = &c;
                if (!L) break;
                const int ndim = backlog.front()->md->geom.ndim, half = backlog.front()->md->half;
                std::vector<EJob*> group, rest;
                for (EJob* j : backlog) (j->md->geom.ndim == ndim && j->md->half == half ? group : rest).push_back(j);
                backlog.swap(rest);
                // one split launch at a time: its teams wait only for their
                // own work-groups, which wait only for finite kernels
                bool split_ok = true;
                for (const TeamLaunch& c : launches) split_ok = split_ok && (c.jobs.empty() || !c.split);
                const wf_status st = team_launch(*L, group, ndim, half, cus, split_ok);
                if (st != WF_OK) {
                    (void)hipStreamSynchronize(L->s);
                    for (EJob* j : group) finish(j, st);
                } else {
                    L->jobs.swap(group);
                }
            }
        } catch (...) {
            // a host allocation failed: settle the launches, fail the rest
            set_thread_staging(nullptr);
            for (TeamLaunch& L : launches) {
                (void)hipStreamSynchronize(L.s);
                std::vector<EJob*> done_jobs;
                done_jobs.swap(L.jobs);
                for (EJob* j : done_jobs) finish(j, WF_OK);
            }
            (void)hipStreamSynchronize(s_setup);
            const wf_status st = fail(WF_E_NOMEM, "host allocation failed while serving");
            std::vector<EJob*> rest;
            rest.swap(backlog);
            rest.insert(rest.end(), pend.begin(), pend.end());
            pend.clear();
            for (; k < fresh.size(); ++k)
                if (std::find(rest.begin(), rest.end(), fresh[k]) == rest.end()) rest.push_back(fresh[k]);
            for (EJob* j : rest) finish(j, st);
        }
    }
    for (TeamLaunch& L : launches) {
        if (L.s) (void)hipStreamSynchronize(L.s);
        if (L.host) (void)hipHostFree(L.host);
        L.dev.reset();
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.s) (void)hipStreamDestroy(L.s);
    }
    if (s_setup) (void)hipStreamSynchronize(s_setup);
    if (staging.base) (void)hipHostFree(staging.base);
    if (host3) (void)hipHostFree(host3);
    if (s_setup) (void)hipStreamDestroy(s_setup);
    set_thread_arena(nullptr);
}

extern "C" {

wf_status wf_engine_create(int64_t hbm_budget_bytes, int max_slots, wf_engine** out) {
    try {
        if (!out) return fail(WF_E_ARG, "out is NULL");
        *out = nullptr;
        if (hbm_budget_bytes < ((int64_t)64 << 20)) return fail(WF_E_ARG, "budget below 64 MiB");
        if (max_slots < 1) return fail(WF_E_ARG, "max_slots must be >= 1");
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(WF_E_HIP, "hipMemGetInfo");
        if (hbm_budget_bytes > (int64_t)fr) return fail(WF_E_BUDGET, "budget exceeds free device memory");
        wf_engine* e = new wf_engine();
        e->arena = arena_create(hbm_budget_bytes);
        if (!e->arena) {
            delete e;
            return WF_E_NOMEM;
        }
        (void)hipGetDevice(&e->device);
        e->budget = hbm_budget_bytes;
        e->max_slots = max_slots;
        if (const char* t = std::getenv("WAVEFD_TEAMS")) e->teams_on = t[0] != '0';
        for (int i = 0; i < kWorkers; ++i) e->threads.emplace_back([e] { e->worker(); });
        e->threads.emplace_back([e] { e->batcher(); });
        e->threads.emplace_back([e] { e->teams(); });
        *out = e;
        return WF_OK;
    } catch (...) {
        return fail(WF_E_NOMEM, "engine creation failed");
    }
}

wf_status wf_engine_submit(wf_engine* e, const wf_request* r, uint64_t* ticket) {
    return wf_engine_submit_on(e, r, nullptr, 0, ticket);
}

wf_status wf_engine_submit_on(wf_engine* e, const wf_request* r, void* stream, int ordered,
                              uint64_t* ticket) {
    try {
        if (!e || !r || !ticket) return fail(WF_E_ARG, "NULL argument");
        wf_status st = check_geom(&r->geom);
        if (st != WF_OK) return st;
        if (r->kind != WF_REQ_FORWARD && r->kind != WF_REQ_GRADIENT) return fail(WF_E_ARG, "unknown request kind");
        if (!r->m_dev) return fail(WF_E_ARG, "m is NULL");
        if (r->nt < 1 || r->nsrc < 0 || r->nrec < 0) return fail(WF_E_ARG, "bad nt or point counts");
        if (!(r->dt > 0.0)) return fail(WF_E_ARG, "dt must be > 0");
        if ((r->nsrc > 0 && (!r->src_xyz || !r->src_wav)) || (r->nrec > 0 && (!r->rec_xyz)))
            return fail(WF_E_ARG, "missing source or receiver arrays");
        if (r->kind == WF_REQ_FORWARD && r->nrec > 0 && !r->rec_out) return fail(WF_E_ARG, "rec_out is NULL");
        if (r->kind == WF_REQ_GRADIENT && (!r->grad_out || (r->nrec > 0 && !r->d_obs)))
            return fail(WF_E_ARG, "gradient requests need grad_out and d_obs");
        EJob* j = new EJob();
        j->rq = *r;
        const int D = r->geom.ndim;
        if (r->nsrc > 0) j->src.assign(r->src_xyz, r->src_xyz + (size_t)r->nsrc * D);
        if (r->nrec > 0) j->rec.assign(r->rec_xyz, r->rec_xyz + (size_t)r->nrec * D);
        j->rq.src_xyz = nullptr;
        j->rq.rec_xyz = nullptr;
        st = footprint(r, j->src.data(), j->rec.data(), e->budget, j);
        if (st == WF_OK && ordered) {
            // the engine's work on this request waits for what the caller has
            // queued on `stream` so far (its inputs), with no host wait
            st = hip_check(hipEventCreateWithFlags(&j->ready, hipEventDisableTiming), "event");
            if (st == WF_OK)
                st = hip_check(hipEventRecord(j->ready, reinterpret_cast<hipStream_t>(stream)), "event record");
        }
        if (st != WF_OK) {
            delete j;
            return st;
        }
        std::lock_guard<std::mutex> lk(e->mu);
        j->ticket = e->next_ticket++;
        *ticket = j->ticket;
        e->pending.push_back(j);
        e->admit();
        return WF_OK;
    } catch (...) {
        return fail(WF_E_NOMEM, "submit failed");
    }
}

wf_status wf_engine_request_bytes(const wf_request* r, int64_t budget, int64_t* bytes) {
    try {
        if (!r || !bytes) return fail(WF_E_ARG, "NULL argument");
        wf_status st = check_geom(&r->geom);
        if (st != WF_OK) return st;
        if (r->nt < 1 || r->nsrc < 0 || r->nrec < 0) return fail(WF_E_ARG, "bad nt or point counts");
        if ((r->nsrc > 0 && !r->src_xyz) || (r->nrec > 0 && !r->rec_xyz))
            return fail(WF_E_ARG, "missing coordinates");
        if (budget <= 0) return fail(WF_E_ARG, "budget must be > 0");
        EJob j;
        (void)footprint(r, r->src_xyz, r->rec_xyz, budget, &j);   // WF_E_BUDGET still sets j.foot
        clear_error();
        *bytes = j.foot;
        return WF_OK;
    } catch (...) {
        return fail(WF_E_NOMEM, "host allocation failed");
    }
}

wf_status wf_engine_poll(wf_engine* e, uint64_t* done_tickets, wf_status* done_status, int cap,
                         int* n_done, int wait_ms) {
    if (!e || !n_done || cap < 0 || (cap > 0 && (!done_tickets || !done_status)))
        return fail(WF_E_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(e->mu);
    if (wait_ms > 0 && e->done.empty())
        e->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !e->done.empty(); });
    int n = 0;
    while (n < cap && !e->done.empty()) {
        done_tickets[n] = e->done.front().first;
        done_status[n] = e->done.front().second;
        e->done.pop_front();
        ++n;
    }
    *n_done = n;
    return WF_OK;
}

wf_status wf_engine_stats(const wf_engine* ce, int64_t* queued, int64_t* running, int64_t* completed,
                          int64_t* bytes_in_use) {
    if (!ce) return fail(WF_E_ARG, "engine is NULL");
    wf_engine* e = const_cast<wf_engine*>(ce);
    std::lock_guard<std::mutex> lk(e->mu);
    if (queued) *queued = (int64_t)e->pending.size();
    if (running) *running = e->running;
    if (completed) *completed = e->completed;
    if (bytes_in_use) *bytes_in_use = arena_used(e->arena);
    return WF_OK;
}

wf_status wf_engine_paths(const wf_engine* ce, int64_t* teams, int64_t* batched, int64_t* workers) {
    if (!ce) return fail(WF_E_ARG, "engine is NULL");
    wf_engine* e = const_cast<wf_engine*>(ce);
    std::lock_guard<std::mutex> lk(e->mu);
    if (teams) *teams = e->served[0];
    if (batched) *batched = e->served[1];
    if (workers) *workers = e->served[2];
    return WF_OK;
}

wf_status wf_engine_destroy(wf_engine* e) {
    if (!e) return WF_OK;
    {
        // every submitted request runs to completion first
        std::unique_lock<std::mutex> lk(e->mu);
        e->cv_done.wait(lk, [&] { return e->pending.empty() && e->running == 0; });
        e->stop = true;
        e->cv_work.notify_all();
    }
    for (auto& t : e->threads) t.join();
    arena_destroy(e->arena);
    for (EJob* j : e->pending) delete j;
    delete e;
    return WF_OK;
}

}  // extern "C"
