// Time loops: forward modelling, its exact adjoint, and the adjoint-state
// gradient with store-all or revolve checkpointing.
//
// Time indexing (nt samples, nt - 1 updates):
//   forward  step n = 0..nt-2: u^{n+1} = S(u^n, u^{n-1}); u^{n+1} += (dt^2/a) P_s^T q^n;
//            d^{n+1} = P_r u^{n+1}; d^0 = 0.
//   adjoint  step n = nt-2..0: v^n = S(v^{n+1}, v^{n+2}); v^n += (dt^2/a) P_r^T y^{n+1};
//            x^n = P_s v^n; x^{nt-1} = 0.
// S is the fused update of the kernels; the adjoint uses the very same S
// because the Laplacian is symmetric and the damping weights a, b are
// diagonal (the transpose of the block lower-triangular A(m), Section
// "Temporal discretization").
// Gradient: g = - sum_{j=1}^{nt-1} u^j (v^{j-1} - 2 v^j + v^{j+1}) / dt^2; the
// term j = n+1 is accumulated by the adjoint step n, inside the stencil kernel
// for the pre-injection v^n and by the injection kernel for the injected part.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace wf {

namespace {

#define WF_TRY(expr)                         \
    do {                                     \
        wf_status st__ = (expr);             \
        if (st__ != WF_OK) return st__;      \
    } while (0)

// Queue-depth limit of the calling thread's time loops (0: none).
thread_local int t_throttle = 0;
struct ThrottleState {
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool armed[2] = {false, false};
    int64_t count = 0;
    ~ThrottleState() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};
thread_local ThrottleState t_thr;

// After every step launch: every t_throttle launches, wait on the host for
// the event recorded t_throttle launches before, then record a new one.
wf_status throttle_tick(hipStream_t s) {
    if (t_throttle <= 0) return WF_OK;
    if (++t_thr.count % t_throttle != 0) return WF_OK;
    const int k = (int)((t_thr.count / t_throttle) & 1);
    if (!t_thr.ev[k])
        WF_TRY(hip_check(hipEventCreateWithFlags(&t_thr.ev[k], hipEventDisableTiming), "event"));
    if (t_thr.armed[k]) WF_TRY(hip_check(hipEventSynchronize(t_thr.ev[k]), "throttle wait"));
    WF_TRY(hip_check(hipEventRecord(t_thr.ev[k], s), "event"));
    t_thr.armed[k] = true;
    return WF_OK;
}

wf_status step(StepParams& p, const Model& md, const float* cur, const float* old, float* out,
               int mode, float* grad, const float* ufwd, hipStream_t s) {
    p.cur = cur;
    p.old = old;
    p.out = out;
    p.grad = grad;
    p.ufwd = ufwd;
    count_step_launch(mode);
    {
        ProfScope prof(WF_KERNEL_STEP, s);
        WF_TRY(hip_check(launch_step(p, md.geom.ndim, md.half, mode, s), "stencil launch"));
    }
    return throttle_tick(s);
}

wf_status inject(const Model& md, const PointSet& ps, const float* vals, float* field, float* grad,
                 const float* ufwd, const StepParams& sp, hipStream_t s) {
    if (ps.nnodes == 0) return WF_OK;
    InjectParams ip;
    ip.field = field;
    ip.kap = md.kap();
    ip.off = ps.d_noff.as<int64_t>();
    ip.eta = ps.d_neta.f();
    ip.seg = ps.d_seg.as<int>();
    ip.pt = ps.d_ept.as<int>();
    ip.w = ps.d_ew.f();
    ip.vals = vals;
    ip.grad = grad;
    ip.ufwd = ufwd;
    ip.nnodes = ps.nnodes;
    ip.inv2dt = sp.inv2dt;
    ip.idt2 = sp.idt2;
    ProfScope prof(WF_KERNEL_INJECT, s);
    return hip_check(launch_inject(ip, s), "inject launch");
}

wf_status sample(const PointSet& ps, const float* field, float* out, hipStream_t s) {
    if (ps.npts == 0) return WF_OK;
    ProfScope prof(WF_KERNEL_SAMPLE, s);
    return hip_check(launch_sample(field, ps.d_off.as<int64_t>(), ps.d_w.f(), ps.npts, ps.K, out, s),
                     "sample launch");
}

// Sources (or receivers in the adjoint) injected by the step kernel itself:
// the per-step increments of every node are computed once per call, and the
// owning thread adds its node's increment before storing the plane. Falls
// back to the separate injection kernel when a block owns more nodes than it
// can stage.
struct Injector {
    const PointSet* ps = nullptr;
    const FusedInj* fz = nullptr;
    const float* vals = nullptr;
    const float* inc = nullptr;

    IncParams ip{};
    // host side: tables and buffers (synchronous work, never captured)
    // geom: the thread layout of another kernel than p's single-update launch
    wf_status plan(Model& md, const PointSet& set, const StepParams& p, const float* series,
                   int nrows, DevBuf& buf, hipStream_t s, const InjGeom* geom = nullptr) {
        ps = &set;
        vals = series;
        fz = nullptr;
        if (set.nnodes == 0) return WF_OK;
        if (!fused_injection_disabled()) {
            if (geom)
                WF_TRY(set.fused(md.L, *geom, &fz));
            else
                WF_TRY(set.fused(md.L, p, &fz));
            if (!fz->ok) fz = nullptr;
        }
        if (!fz) return WF_OK;
        const int64_t need = (int64_t)nrows * fz->nnodes * 4;
        if (buf.bytes < need) {
            WF_TRY(hip_check(hipStreamSynchronize(s), "sync"));   // buffer may be in use
            WF_TRY(buf.alloc(need));
        }
        ip.inc = buf.f();
        ip.kap = md.kap();
        ip.off = fz->off.as<int64_t>();
        ip.eta = fz->eta.f();
        ip.seg = fz->seg.as<int>();
        ip.pt = fz->pt.as<int>();
        ip.w = fz->w.f();
        ip.vals = series;
        ip.nnodes = fz->nnodes;
        ip.npts = set.npts;
        ip.nrows = nrows;
        ip.inv2dt = p.inv2dt;
        inc = buf.f();
        return WF_OK;
    }
    // device side: the increments of every step
    wf_status enqueue(hipStream_t s) const {
        if (!fz) return WF_OK;
        return hip_check(launch_increments(ip, s), "increments");
    }
    wf_status prepare(Model& md, const PointSet& set, const StepParams& p, const float* series,
                      int nrows, DevBuf& buf, hipStream_t s) {
        WF_TRY(plan(md, set, p, series, nrows, buf, s));
        return enqueue(s);
    }
    // configure the step that injects row `row`
    void configure(StepParams& p, int64_t row) const {
        p.inj_blk = nullptr;
        if (!fz) return;
        p.inj_blk = fz->blk.as<int>();
        p.inj_thr = fz->thr.as<int2>();
        p.inj_x = fz->x.as<int>();
        p.inj_inc = reinterpret_cast<const float4*>(inc + row * fz->nnodes);
    }
    // after the step: the separate kernel when not fused
    wf_status after(const Model& md, int64_t row, float* field, float* grad, const float* ufwd,
                    const StepParams& p, hipStream_t s) const {
        if (fz || !ps || ps->nnodes == 0) return WF_OK;
        return inject(md, *ps, vals + row * ps->npts, field, grad, ufwd, p, s);
    }
};

// Receivers spread evenly over the blocks of the (already planned) launch.
void set_sampling(StepParams& p, const PointSet* ps, float* out) {
    if (!ps || ps->npts == 0 || !out) {
        p.smp_out = nullptr;
        p.smp_per = 0;
        p.smp_n = 0;
        return;
    }
    p.smp_off = ps->d_off.as<int64_t>();
    p.smp_w = ps->d_w.f();
    p.smp_out = out;
    p.smp_n = ps->npts;
    p.smp_per = (int)(((int64_t)ps->npts + p.nblocks - 1) / p.nblocks);
}


}  // namespace

// Time loops as HIP graphs: the host prepares everything first (plans,
// tables, buffers); the enqueue phase (fills, increments, every step, the last
// sample) is then either issued directly or captured once and replayed. A
// signature (every pointer and size the loop bakes in) runs eagerly the first
// time, is captured on its next call while still among the recent ones, and
// replays from then on; a few captured loops are kept per model. Graphs run
// on the model's own stream, ordered after and before the caller's stream
// with events.
namespace {

int64_t bits_of(double x) {
    int64_t b;
    std::memcpy(&b, &x, sizeof b);
    return b;
}

// Off unless asked for: on ROCm 7.x a replayed kernel node costs 0.5-1 us
// more than the same launch issued to a stream (measured from 2e4 to 4e7
// nodes), so graphs pay only where a caller needs the loop as one unit.
std::atomic<int>& graph_switch() {
    static std::atomic<int> on{[] {
        const char* e = std::getenv("WAVEFD_GRAPH");
        return (e && e[0] == '1') ? 1 : 0;
    }()};
    return on;
}

bool graphs_enabled() { return graph_switch().load(std::memory_order_relaxed) != 0; }

wf_status launch_graph(Model& md, Model::GraphEntry& e, hipStream_t s) {
    e.tick = ++md.graph_tick;
    WF_TRY(hip_check(hipEventRecord(md.ev_in, s), "event"));
    WF_TRY(hip_check(hipStreamWaitEvent(md.gstream, md.ev_in, 0), "wait"));
    WF_TRY(hip_check(hipGraphLaunch(e.exec, md.gstream), "graph launch"));
    ++md.graph_launches;
    WF_TRY(hip_check(hipEventRecord(md.ev_out, md.gstream), "event"));
    return hip_check(hipStreamWaitEvent(s, md.ev_out, 0), "wait");
}

// Replay a captured loop with this signature; else capture it if the
// signature ran eagerly in one of the last calls; else run it eagerly.
template <class F>
wf_status run_maybe_graph(Model& md, const GraphKey& key, hipStream_t s, F&& enqueue) {
    if (!graphs_enabled() || profiling_active() || t_throttle > 0 || thread_scratch_active()) return enqueue(s);
    for (Model::GraphEntry& e : md.graphs)
        if (e.key == key) return launch_graph(md, e, s);
    auto it = std::find(md.seen.begin(), md.seen.end(), key);
    if (it == md.seen.end()) {
        if (md.seen.size() >= Model::kMaxSeen) md.seen.erase(md.seen.begin());
        md.seen.push_back(key);
        return enqueue(s);
    }
    md.seen.erase(it);
    WF_TRY(md.ensure_graph_stream());
    if (md.graphs.size() >= Model::kMaxGraphs) {   // evict the least recently used
        auto lru = std::min_element(md.graphs.begin(), md.graphs.end(),
                                    [](const Model::GraphEntry& a, const Model::GraphEntry& b) {
                                        return a.tick < b.tick;
                                    });
        WF_TRY(hip_check(hipStreamSynchronize(md.gstream), "sync"));
        (void)hipGraphExecDestroy(lru->exec);
        (void)hipGraphDestroy(lru->graph);
        md.graphs.erase(lru);
    }
    // capture on the model's stream, ordered after the caller's earlier work
    WF_TRY(hip_check(hipEventRecord(md.ev_in, s), "event"));
    WF_TRY(hip_check(hipStreamWaitEvent(md.gstream, md.ev_in, 0), "wait"));
    WF_TRY(hip_check(hipStreamBeginCapture(md.gstream, hipStreamCaptureModeThreadLocal), "begin capture"));
    const wf_status st = enqueue(md.gstream);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(md.gstream, &g);
    if (st != WF_OK || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != WF_OK ? st : hip_check(ce, "end capture");
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_check(ie, "graph instantiate");
    }
    Model::GraphEntry e;
    e.key = key;
    e.graph = g;
    e.exec = ex;
    md.graphs.push_back(e);
    return launch_graph(md, md.graphs.back(), s);
}

}  // namespace

void set_graphs_enabled(bool on) { graph_switch().store(on ? 1 : 0); }

namespace {
// 0 off, 1 where the two-update kernel was measured faster, 2 wherever compiled
std::atomic<int>& two_step_switch() {
    static std::atomic<int> mode{[] {
        const char* e = std::getenv("WAVEFD_TWO_STEP");
        if (e && e[0] == '0') return 0;
        if (e && e[0] == '2') return 2;
        return 1;
    }()};
    return mode;
}
}  // namespace

void set_two_step_mode(int mode) { two_step_switch().store(std::min(2, std::max(0, mode))); }

bool fused_injection_disabled() { return std::getenv("WAVEFD_NO_FUSED_INJECT") != nullptr; }

void set_thread_throttle(int steps) {
    t_throttle = std::max(0, steps);
    t_thr.count = 0;
    t_thr.armed[0] = t_thr.armed[1] = false;
}

namespace {

// Two updates per launch (3D, compiled orders) for loops of two updates or
// more, where the mode allows it; calls that allocate from an arena or a
// fixed scratch keep one. `pts` are the points injected (sources of a
// forward loop, receivers of an adjoint one), `smp` the points sampled.
struct TwoStep {
    bool on = false;
    Step2Params p2{};
    Injector inj[2];   // [0]: the first update's extended tile, [1]: the second's inner tile
    wf_status plan(Model& md, const StepParams& p, int nt, const PointSet& pts, const float* series,
                   const PointSet& smp, hipStream_t s) {
        const Layout& L = md.L;
        const int mode = two_step_switch().load(std::memory_order_relaxed);
        on = nt >= 3 && step2_supported(L.ndim, md.half) &&
             (mode == 2 || (mode == 1 && step2_preferred(L.ndim, md.half, L.npoints))) &&
             !thread_arena_active() && !thread_scratch_active() &&
             !(pts.nnodes > 0 && fused_injection_disabled());
        if (!on) return WF_OK;
        p2.kap = p.kap;
        p2.etax = p.etax;
        p2.etay = p.etay;
        p2.etaz = p.etaz;
        p2.nx = p.nx;
        p2.ny = p.ny;
        p2.nz = p.nz;
        p2.sx = p.sx;
        p2.sy = p.sy;
        p2.c0 = p.c0;
        std::copy(p.wx, p.wx + kMaxHalf + 1, p2.wx);
        std::copy(p.wy, p.wy + kMaxHalf + 1, p2.wy);
        std::copy(p.wz, p.wz + kMaxHalf + 1, p2.wz);
        p2.inv2dt = p.inv2dt;
        step2_plan(p2, L.ndim, md.half, 0);
        if (pts.nnodes > 0) {
            const int M = md.half, hz = step2_ext_cols(M), my = L.ndim == 3 ? M : 0;
            InjGeom g;
            g.tz = 4 * (step2_cols(L.ndim == 3) - 2 * hz);
            g.ty = p2.by;
            g.bz = step2_cols(L.ndim == 3);
            g.nt = step2_threads(L.ndim, M, p2.by);
            g.ntz = p2.ntz;
            g.nty = p2.nty;
            g.cx = p2.cx;
            g.nchunks = p2.nchunks;
            g.nblocks = p2.nblocks;
            g.cap = step2_inj_cap(L.ndim == 3);
            g.tag = 2;
            InjGeom ge = g;   // first update: the extended tile and chunk
            ge.ey = my;
            ge.ez4 = hz;
            ge.ex = M;
            InjGeom gi = g;   // second update: the inner tile, numbered in the extended one
            gi.oy = my;
            gi.oz4 = hz;
            WF_TRY(inj[0].plan(md, pts, p, series, nt, md.d_inc[1], s, &ge));
            WF_TRY(inj[1].plan(md, pts, p, series, nt, md.d_inc[2], s, &gi));
            on = inj[0].fz && inj[1].fz;
            if (!on) return WF_OK;
        }
        if (smp.npts > 0) {
            p2.smp_off = smp.d_off.as<int64_t>();
            p2.smp_w = smp.d_w.f();
            p2.smp_n = smp.npts;
            p2.smp_per = (int)(((int64_t)smp.npts + p2.nblocks - 1) / p2.nblocks);
        }
        // without room for the second field pair the loop keeps one update
        // per launch (the same results), rather than failing
        const wf_status st = md.ensure_u2(s);
        if (st == WF_E_NOMEM) {
            clear_error();
            md.d_u2[0].reset();
            md.d_u2[1].reset();
            on = false;
            return WF_OK;
        }
        return st;
    }
    void key(std::vector<int64_t>& v, const Model& md) const {
        v.push_back(on ? 1 : 0);
        if (!on) return;
        for (int64_t x : {(int64_t)p2.cx, (int64_t)(intptr_t)md.u2(0), (int64_t)(intptr_t)md.u2(1),
                          (int64_t)(intptr_t)inj[0].inc, (int64_t)(intptr_t)inj[1].inc,
                          (int64_t)(intptr_t)inj[0].fz, (int64_t)(intptr_t)inj[1].fz})
            v.push_back(x);
    }
    // device side: the increments of every step of both tables
    wf_status enqueue(hipStream_t q) const {
        WF_TRY(inj[0].enqueue(q));
        return inj[1].enqueue(q);
    }
    // one launch: out1 = S(cur, old) + increments of row r1, out2 = S(out1,
    // cur) + those of row r2; samples of cur and old into smp_cur / smp_old
    wf_status launch(const Model& md, const float* cur, const float* old, float* out1, float* out2,
                     int64_t r1, int64_t r2, float* smp_cur, float* smp_old, hipStream_t q) const {
        Step2Params x = p2;
        x.cur = cur;
        x.old = old;
        x.out1 = out1;
        x.out2 = out2;
        x.smp_cur = p2.smp_n > 0 ? smp_cur : nullptr;
        x.smp_old = p2.smp_n > 0 ? smp_old : nullptr;
        const int64_t rows[2] = {r1, r2};
        for (int k = 0; k < 2; ++k) {
            x.inj_blk[k] = nullptr;
            const Injector& ik = inj[k];
            if (!ik.fz) continue;
            x.inj_blk[k] = ik.fz->blk.as<int>();
            x.inj_thr[k] = ik.fz->thr.as<int2>();
            x.inj_x[k] = ik.fz->x.as<int>();
            x.inj_inc[k] = reinterpret_cast<const float4*>(ik.inc + rows[k] * ik.fz->nnodes);
        }
        count_step_launch(kModeCount);
        {
            ProfScope prof(WF_KERNEL_STEP2, q);
            WF_TRY(hip_check(launch_step2(x, md.L.ndim, md.half, q), "two-update launch"));
        }
        return throttle_tick(q);
    }
};

}  // namespace

wf_status run_forward(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                      const PointSet& rec, float* rec_out, float* u_save, int save_every,
                      hipStream_t s, DevBuf* inc_buf) {
    const Layout& L = md.L;
    WF_TRY(md.ensure_kap(dt, s));
    StepParams p;
    md.fill_step(p, dt, false);
    Injector inj;
    WF_TRY(inj.plan(md, src, p, src_wav, nt, inc_buf ? *inc_buf : md.d_inc[0], s));

    TwoStep two;
    WF_TRY(two.plan(md, p, nt, src, src_wav, rec, s));

    GraphKey key;
    key.v = {0, (int64_t)nt, bits_of(dt), src.gen, rec.gen, (int64_t)(intptr_t)src_wav,
             (int64_t)(intptr_t)rec_out, (int64_t)(intptr_t)u_save, save_every, p.cx, p.tile,
             (int64_t)(intptr_t)inj.inc, (int64_t)(intptr_t)inj.fz, (int64_t)(intptr_t)md.u(0),
             (int64_t)(intptr_t)md.u(1), (int64_t)(intptr_t)md.kap()};
    two.key(key.v, md);
    auto enqueue = [&](hipStream_t q) -> wf_status {
        float* A = md.u(0);   // u^n
        float* B = md.u(1);   // u^{n-1}, overwritten by u^{n+1}
        WF_TRY(hip_check(launch_fill(A, L.elems, 0.0f, q), "fill"));
        WF_TRY(hip_check(launch_fill(B, L.elems, 0.0f, q), "fill"));
        if (u_save) WF_TRY(hip_check(launch_fill(u_save, L.npoints, 0.0f, q), "fill"));
        WF_TRY(inj.enqueue(q));
        if (nt == 1 && rec.npts > 0) WF_TRY(hip_check(launch_fill(rec_out, rec.npts, 0.0f, q), "fill"));
        int n = 0;
        if (two.on) {
            // launch at n: u^{n+1} and u^{n+2} from u^n and u^{n-1}; q^n and
            // q^{n+1} injected; d^n and d^{n-1} sampled from the fields it reads
            WF_TRY(two.enqueue(q));
            float* C = md.u2(0);
            float* D = md.u2(1);
            RunSpan span2(q, WF_KERNEL_STEP2_RUN);
            int launches = 0;
            for (; n + 2 < nt; n += 2) {
                float* dc = rec.npts ? rec_out + (int64_t)n * rec.npts : nullptr;
                float* dold = (rec.npts && n >= 1) ? rec_out + (int64_t)(n - 1) * rec.npts : nullptr;
                WF_TRY(two.launch(md, A, B, C, D, n, n + 1, dc, dold, q));
                ++launches;
                if (u_save && (n + 1) % save_every == 0)
                    WF_TRY(hip_check(launch_unpitch(C, u_save + (int64_t)((n + 1) / save_every) * L.npoints,
                                                    L.nx, L.ny, L.nz, L.sx, L.sy, q), "save"));
                if (u_save && (n + 2) % save_every == 0)
                    WF_TRY(hip_check(launch_unpitch(D, u_save + (int64_t)((n + 2) / save_every) * L.npoints,
                                                    L.nx, L.ny, L.nz, L.sx, L.sy, q), "save"));
                std::swap(A, D);   // u^{n+2}
                std::swap(B, C);   // u^{n+1}
            }
            span2.finish(launches);
            // d^{n-1} is in the old field, which the loop below overwrites
            WF_TRY(sample(rec, B, rec_out + (int64_t)(n - 1) * rec.npts, q));
        }
        StepParams ps = p;
        RunSpan span(q);
        int singles = 0;
        for (; n + 1 < nt; ++n) {
            // step n: u^{n+1} from u^n, u^{n-1}; q^n injected; d^n = P_r u^n sampled
            inj.configure(ps, n);
            set_sampling(ps, &rec, rec.npts ? rec_out + (int64_t)n * rec.npts : nullptr);
            WF_TRY(step(ps, md, A, B, B, kModePlain, nullptr, nullptr, q));
            WF_TRY(inj.after(md, n, B, nullptr, nullptr, ps, q));
            if (u_save && (n + 1) % save_every == 0)
                WF_TRY(hip_check(launch_unpitch(B, u_save + (int64_t)((n + 1) / save_every) * L.npoints,
                                                L.nx, L.ny, L.nz, L.sx, L.sy, q), "save"));
            std::swap(A, B);
            ++singles;
        }
        span.finish(singles);
        if (nt > 1) WF_TRY(sample(rec, A, rec_out + (int64_t)(nt - 1) * rec.npts, q));
        return WF_OK;
    };
    return run_maybe_graph(md, key, s, enqueue);
}

wf_status run_adjoint(Model& md, double dt, int nt, const PointSet& rec, const float* rec_in,
                      const PointSet& src, float* src_out, hipStream_t s) {
    const Layout& L = md.L;
    WF_TRY(md.ensure_kap(dt, s));
    StepParams p;
    md.fill_step(p, dt, false);
    Injector inj;
    WF_TRY(inj.plan(md, rec, p, rec_in, nt, md.d_inc[0], s));
    TwoStep two;
    WF_TRY(two.plan(md, p, nt, rec, rec_in, src, s));
    GraphKey key;
    key.v = {1, (int64_t)nt, bits_of(dt), rec.gen, src.gen, (int64_t)(intptr_t)rec_in,
             (int64_t)(intptr_t)src_out, 0, 0, p.cx, p.tile, (int64_t)(intptr_t)inj.inc,
             (int64_t)(intptr_t)inj.fz, (int64_t)(intptr_t)md.u(0), (int64_t)(intptr_t)md.u(1),
             (int64_t)(intptr_t)md.kap()};
    two.key(key.v, md);
    auto enqueue = [&](hipStream_t q) -> wf_status {
        float* A = md.u(0);   // v^{n+1}
        float* B = md.u(1);   // v^{n+2}, overwritten by v^n
        WF_TRY(hip_check(launch_fill(A, L.elems, 0.0f, q), "fill"));
        WF_TRY(hip_check(launch_fill(B, L.elems, 0.0f, q), "fill"));
        WF_TRY(inj.enqueue(q));
        if (nt == 1 && src.npts > 0) WF_TRY(hip_check(launch_fill(src_out, src.npts, 0.0f, q), "fill"));
        int n = nt - 2;
        if (two.on) {
            // launch at n: v^n and v^{n-1} from v^{n+1} and v^{n+2}; y^{n+1}
            // and y^n injected; x^{n+1} and x^{n+2} sampled from the fields it reads
            WF_TRY(two.enqueue(q));
            float* C = md.u2(0);
            float* D = md.u2(1);
            RunSpan span2(q, WF_KERNEL_STEP2_RUN);
            int launches = 0;
            for (; n >= 1; n -= 2) {
                float* xc = src.npts ? src_out + (int64_t)(n + 1) * src.npts : nullptr;
                float* xo = (src.npts && n + 2 <= nt - 1) ? src_out + (int64_t)(n + 2) * src.npts : nullptr;
                WF_TRY(two.launch(md, A, B, C, D, n + 1, n, xc, xo, q));
                ++launches;
                std::swap(A, D);   // v^{n-1}
                std::swap(B, C);   // v^n
            }
            span2.finish(launches);
            // x^{n+2} is in the old field, which the loop below overwrites
            WF_TRY(sample(src, B, src_out + (int64_t)(n + 2) * src.npts, q));
        }
        StepParams ps = p;
        RunSpan span(q);
        int singles = 0;
        for (; n >= 0; --n) {
            // step n: v^n from v^{n+1}, v^{n+2}; y^{n+1} injected; x^{n+1} = P_s v^{n+1} sampled
            inj.configure(ps, n + 1);
            set_sampling(ps, &src, src.npts ? src_out + (int64_t)(n + 1) * src.npts : nullptr);
            WF_TRY(step(ps, md, A, B, B, kModePlain, nullptr, nullptr, q));
            WF_TRY(inj.after(md, n + 1, B, nullptr, nullptr, ps, q));
            std::swap(A, B);
            ++singles;
        }
        span.finish(singles);
        if (nt > 1) WF_TRY(sample(src, A, src_out, q));
        return WF_OK;
    };
    return run_maybe_graph(md, key, s, enqueue);
}

// ---------------------------------------------------------------------------
// gradient
// ---------------------------------------------------------------------------
namespace {

// A pool of pitched field buffers (with zero ghost planes) carved from one
// allocation, zeroed once.
struct FieldPool {
    DevBuf own;
    float* base = nullptr;
    int64_t stride = 0;   // floats per buffer
    int64_t off = 0;      // plane 0 within a buffer
    int count = 0;
    static int64_t bytes_for(const Layout& L, int n) {
        return (int64_t)n * ((L.alloc_elems + 63) / 64 * 64) * 4 + 256;
    }
    // n buffers in `buf` (grown if too small; work enqueued on s before this
    // call may still read the old contents, so growing waits for it). All n
    // are zeroed, unless `clean` says that every ghost plane in `buf` is
    // still zero from an earlier carve (kernels never write ghost planes):
    // then only the first nzero buffers are, the rest being written before
    // they are read.
    wf_status carve(DevBuf& buf, const Layout& L, int n, hipStream_t s, int nzero = -1,
                    bool* clean = nullptr) {
        stride = (L.alloc_elems + 63) / 64 * 64;
        off = L.ghost_off;
        count = n;
        const int64_t need = bytes_for(L, n);
        bool fresh = false;
        if (buf.bytes < need) {
            wf_status st = hip_check(hipStreamSynchronize(s), "sync");
            if (st == WF_OK) {
                buf.reset();
                st = buf.alloc(need);
            }
            if (st != WF_OK) return st;
            fresh = true;
        }
        base = buf.f();
        if (nzero < 0 || !clean) return hip_check(launch_fill(base, need / 4, 0.0f, s), "fill");
        if (fresh || !*clean) {
            WF_TRY(hip_check(launch_fill(base, buf.bytes / 4, 0.0f, s), "fill"));
            *clean = true;
            return WF_OK;
        }
        return hip_check(launch_fill(base, std::min<int64_t>(need / 4, (int64_t)nzero * stride), 0.0f, s),
                         "fill");
    }
    wf_status alloc(const Layout& L, int n, hipStream_t s) { return carve(own, L, n, s); }
    float* at(int i) const { return base + (int64_t)i * stride + off; }
    float* raw(int i) const { return base + (int64_t)i * stride; }   // start of buffer i
};

}  // namespace

namespace {

// Boundary-wavefield reconstruction (Section "Discrete adjoint wave-equation
// and FWI gradient", the alternative to checkpointing it describes): the
// forward sweep stores, per step, only the face slabs around the physical grid
// that its stencil reads; the reverse sweep rebuilds u backward on the physical
// grid next to the adjoint field, with the same update (where eta = 0 it is
// its own time reverse: u^{n-1} = 2 u^n - u^{n+1} + kappa L u^n + the injected
// q^n) and the stored slabs restored after every step. One extra wave solve,
// memory O(surface x nt). The layer itself is not rebuilt (reversing the
// damping is unstable), so the gradient is formed on the physical grid and is
// zero in the layer.
wf_status gradient_boundary(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                            const PointSet& rec, const float* residual, const ObsData* obs, float* G,
                            int64_t held, int64_t budget, hipStream_t s, StepParams& p,
                            StepParams& pi) {
    const Layout& L = md.L;
    const int64_t fb = ((L.alloc_elems + 63) / 64 * 64) * 4;
    const int64_t l = nt - 1;
    const int64_t nrec = rec.npts;
    const StripGeom sg = md.strips();
    const int64_t per = sg.start[sg.nslab];                 // floats per stored step
    const int64_t strip_fields = ((int64_t)nt * per * 4 + fb - 1) / fb;
    int64_t cap = device_free_bytes() + held + md.ws.bytes;
    if (budget > 0) cap = std::min<int64_t>(cap, budget);
    const int64_t need = held + (4 + strip_fields) * fb;
    if (need > cap) return fail(WF_E_BUDGET, "gradient needs %lld bytes, %lld available", (long long)need, (long long)cap);
    // A, B, V1, V2 start at zero; the slabs overwrite ghost planes of the
    // workspace, which the next carve must therefore clear again
    FieldPool pool;
    WF_TRY(pool.carve(md.ws, L, (int)(4 + strip_fields), s, 4, &md.ws_clean));
    md.ws_clean = false;
    float* A = pool.at(0);    // u^n in the forward sweep, u^{n+1} in the reverse sweep
    float* B = pool.at(1);
    float* V1 = pool.at(2);   // v^{n+1}
    float* V2 = pool.at(3);   // v^{n+2}, overwritten by v^n
    float* strips = pool.raw(4);   // row n: the slabs of u^n (row 0: u^0 = 0)
    WF_TRY(hip_check(launch_fill(strips, per, 0.0f, s), "fill"));

    Injector qinj, rinj;
    WF_TRY(qinj.prepare(md, src, p, src_wav, nt, md.d_inc[0], s));
    if (!obs) WF_TRY(rinj.prepare(md, rec, pi, residual, nt, md.d_inc[1], s));

    // forward sweep: u^{n+1} over u^{n-1}, then its slabs into row n+1
    for (int64_t n = 0; n < l; ++n) {
        qinj.configure(p, n);
        set_sampling(p, obs ? &rec : nullptr, (obs && nrec) ? obs->d_pred + n * nrec : nullptr);
        WF_TRY(step(p, md, A, B, B, kModePlain, nullptr, nullptr, s));
        WF_TRY(qinj.after(md, n, B, nullptr, nullptr, p, s));
        WF_TRY(hip_check(launch_strip(B, strips + (n + 1) * per, sg, 0, s), "save strips"));
        std::swap(A, B);
    }
    // now A = u^{nt-1}, B = u^{nt-2}
    if (obs) {
        if (nrec > 0) {
            WF_TRY(sample(rec, A, obs->d_pred + l * nrec, s));
            WF_TRY(hip_check(launch_residual(obs->d_pred, obs->d_obs, obs->resid, (int64_t)nt * nrec,
                                             obs->partial, s), "residual"));
        }
        WF_TRY(rinj.prepare(md, rec, pi, obs->resid, nt, md.d_inc[1], s));
    }
    set_sampling(p, nullptr, nullptr);
    for (int64_t n = l - 1; n >= 0; --n) {
        // adjoint step n with imaging of term j = n+1 (A = u^{n+1})
        rinj.configure(pi, n + 1);
        WF_TRY(step(pi, md, V1, V2, V2, kModeImaging, G, A, s));
        WF_TRY(rinj.after(md, n + 1, V2, G, A, pi, s));
        std::swap(V1, V2);
        if (n >= 2) {
            // u^{n-1} = 2 u^n - u^{n+1} + kappa L u^n + q^n's injection, over u^{n+1}
            qinj.configure(p, n);
            WF_TRY(step(p, md, B, A, A, kModePlain, nullptr, nullptr, s));
            WF_TRY(qinj.after(md, n, A, nullptr, nullptr, p, s));
            WF_TRY(hip_check(launch_strip(A, strips + (n - 1) * per, sg, 1, s), "restore strips"));
        }
        std::swap(A, B);   // A = u^n for the next adjoint step
    }
    int b0[3], b1[3];
    md.interior(b0, b1);
    WF_TRY(hip_check(launch_mask_box(G, L.nx, L.ny, L.nz, L.sx, L.sy, b0[0], b1[0], b0[1], b1[1], b0[2],
                                     b1[2], s), "mask"));
    return hip_check(hipStreamSynchronize(s), "sync");
}

// One shot's adjoint-state gradient added into the pitched accumulator G.
// With `obs`, the residual is formed inside the call: the first forward sweep
// samples d = P_r u into obs->d_pred, and before the first reverse step
// r = d - d_obs goes to obs->resid with the FP64 partial sums of |r|^2 in
// obs->partial (two wave solves per shot). Otherwise `residual` is given.
// `held` bytes (the accumulator and the record scratch, allocated by the
// caller) count against the budget.
wf_status gradient_core(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                        const PointSet& rec, const float* residual, const ObsData* obs, float* G,
                        int64_t held, int n_ck, int64_t budget, hipStream_t s) {
    const Layout& L = md.L;
    const int64_t fb = ((L.alloc_elems + 63) / 64 * 64) * 4;
    WF_TRY(md.ensure_kap(dt, s));
    StepParams p, pi;
    md.fill_step(p, dt);
    md.fill_step(pi, dt, kModeImaging);
    const int64_t l = nt - 1;                     // adjoint steps n = 0..nt-2
    const int64_t nrec = rec.npts;
    if (l <= 0) {
        // one sample: u^0 = 0, so d^0 = 0 and the gradient has no term
        if (obs && nrec > 0) {
            WF_TRY(hip_check(launch_fill(obs->d_pred, nrec, 0.0f, s), "fill"));
            WF_TRY(hip_check(launch_residual(obs->d_pred, obs->d_obs, obs->resid, nrec, obs->partial, s),
                             "residual"));
        }
        return WF_OK;
    }
    if (n_ck == -2)
        return gradient_boundary(md, dt, nt, src, src_wav, rec, residual, obs, G, held, budget, s, p, pi);
    // memory plan: adjoint pair + what the caller holds (accumulator, record
    // scratch) plus either every forward field (store-all: nt fields incl. one
    // zero field) or a revolve pool of 2 s + 3 fields
    int64_t cap = device_free_bytes() + held + md.ws.bytes;   // the workspace is reused
    if (budget > 0) cap = std::min<int64_t>(cap, budget);
    const int64_t fixed = 2 * fb + held;
    bool store_all = false;
    int snaps = n_ck;
    if (n_ck == -1) {
        store_all = true;
    } else if (n_ck == 0) {
        const int64_t all_bytes = fixed + (int64_t)nt * fb;
        if (all_bytes <= cap) store_all = true;
        else {
            snaps = (int)std::min<int64_t>((cap - fixed - 3 * fb) / (2 * fb), l);
            if (snaps < 1) return fail(WF_E_BUDGET, "gradient needs at least %lld bytes", (long long)(fixed + 5 * fb));
        }
    } else if (n_ck < -1) {
        return fail(WF_E_ARG, "n_checkpoints must be >= -2");
    }
    if (!store_all) snaps = (int)std::min<int64_t>(snaps, l);
    const int nbuf = store_all ? nt : 2 * snaps + 3;
    const int64_t need = fixed + (int64_t)nbuf * fb;
    if (need > cap) return fail(WF_E_BUDGET, "gradient needs %lld bytes, %lld available", (long long)need, (long long)cap);

    // one carve of the model's workspace (kept for the next call: allocating
    // tens of GB again costs seconds) holds the pool and the adjoint pair
    // the adjoint pair and the first two forward buffers (u^0 = u^{-1} = 0)
    // start at zero; every other buffer is written before it is read
    FieldPool pool;
    WF_TRY(pool.carve(md.ws, L, nbuf + 2, s, 4, &md.ws_clean));
    float* V1 = pool.at(0);   // v^{n+1}
    float* V2 = pool.at(1);   // v^{n+2}, overwritten by v^n
    auto F = [&](int i) { return pool.at(2 + i); };   // forward buffer i
    Injector qinj, rinj;   // sources in forward steps, residual in adjoint steps
    WF_TRY(qinj.prepare(md, src, p, src_wav, nt, md.d_inc[0], s));
    bool resid_ready = obs == nullptr;
    if (resid_ready) WF_TRY(rinj.prepare(md, rec, pi, residual, nt, md.d_inc[1], s));
    int64_t next_row = 0;   // first record row not yet sampled (observed-data mode)

    // forward step n: u^{n+1} into `out` from u^n, u^{n-1}, injecting q^n;
    // on the first sweep (observed-data mode) it also samples d^n = P_r u^n
    auto forward_step = [&](int64_t n, const float* cur, const float* old, float* out) -> wf_status {
        qinj.configure(p, n);
        if (obs && n == next_row) {
            set_sampling(p, &rec, nrec ? obs->d_pred + n * nrec : nullptr);
            ++next_row;
        } else {
            set_sampling(p, nullptr, nullptr);
        }
        WF_TRY(step(p, md, cur, old, out, kModePlain, nullptr, nullptr, s));
        return qinj.after(md, n, out, nullptr, nullptr, p, s);
    };
    // before the first reverse step: the last record row and the residual
    auto form_residual = [&](const float* u_last) -> wf_status {
        if (resid_ready) return WF_OK;
        if (next_row != l) return fail(WF_E_STATE, "record incomplete before the reverse sweep");
        if (nrec > 0) {
            WF_TRY(sample(rec, u_last, obs->d_pred + l * nrec, s));
            WF_TRY(hip_check(launch_residual(obs->d_pred, obs->d_obs, obs->resid, (int64_t)nt * nrec,
                                             obs->partial, s), "residual"));
        }
        WF_TRY(rinj.prepare(md, rec, pi, obs->resid, nt, md.d_inc[1], s));
        resid_ready = true;
        return WF_OK;
    };
    // adjoint step n with imaging of term j = n+1 (u^{n+1} given)
    auto reverse_step = [&](int64_t n, const float* u_np1) -> wf_status {
        WF_TRY(form_residual(u_np1));
        rinj.configure(pi, n + 1);
        WF_TRY(step(pi, md, V1, V2, V2, kModeImaging, G, u_np1, s));
        WF_TRY(rinj.after(md, n + 1, V2, G, u_np1, pi, s));
        std::swap(V1, V2);
        return WF_OK;
    };

    if (store_all) {
        // buffer 0 is zero and stands for both u^0 and u^{-1}; buffer j holds u^j
        for (int64_t n = 0; n + 1 < nt; ++n) {
            const float* cur = F((int)n);
            const float* old = F((int)std::max<int64_t>(n - 1, 0));
            WF_TRY(forward_step(n, cur, old, F((int)(n + 1))));
        }
        for (int64_t n = nt - 2; n >= 0; --n) WF_TRY(reverse_step(n, F((int)(n + 1))));
    } else {
        std::vector<RevolveAction> acts;
        WF_TRY(revolve_schedule(l, snaps, acts));
        // state x_i = (u^{i+1}, u^i) held in buffers (bn, bo); pinned buffers
        // belong to snapshot slots and are never written
        std::vector<int> pin(nbuf, 0);
        std::vector<std::pair<int, int>> slot(snaps, {-1, -1});
        int bn = 0, bo = 1;
        auto take_free = [&](int avoid1, int avoid2) -> int {
            for (int b = 0; b < nbuf; ++b)
                if (pin[b] == 0 && b != avoid1 && b != avoid2) return b;
            return -1;
        };
        // x_0: u^0 = u^{-1} = 0 (the pool starts zeroed), one forward step injecting q^0
        WF_TRY(forward_step(0, F(0), F(1), F(1)));
        bn = 1;
        bo = 0;
        int64_t pos = 0;
        for (const RevolveAction& a : acts) {
            switch (a.kind) {
                case RevolveAction::ADVANCE:
                    if (a.at != pos) return fail(WF_E_STATE, "revolve: advance from %lld at %lld", (long long)a.at, (long long)pos);
                    for (int64_t i = pos; i < a.arg; ++i) {
                        // forward step F_{i+1}: u^{i+2} from u^{i+1} (bn), u^i (bo), q^{i+1}
                        int out = pin[bo] == 0 ? bo : take_free(bn, bo);
                        if (out < 0) return fail(WF_E_STATE, "revolve: buffer pool exhausted");
                        WF_TRY(forward_step(i + 1, F(bn), F(bo), F(out)));
                        bo = bn;
                        bn = out;
                    }
                    pos = a.arg;
                    break;
                case RevolveAction::TAKESHOT:
                    if (a.at != pos) return fail(WF_E_STATE, "revolve: snapshot out of place");
                    slot[(size_t)a.arg] = {bn, bo};
                    ++pin[bn];
                    ++pin[bo];
                    break;
                case RevolveAction::RESTORE:
                    bn = slot[(size_t)a.arg].first;
                    bo = slot[(size_t)a.arg].second;
                    pos = a.at;
                    break;
                case RevolveAction::REVERSE:
                    if (a.at != pos) return fail(WF_E_STATE, "revolve: reverse step out of place");
                    WF_TRY(reverse_step(a.at, F(bn)));
                    break;
                case RevolveAction::FREE:
                    --pin[slot[(size_t)a.arg].first];
                    --pin[slot[(size_t)a.arg].second];
                    slot[(size_t)a.arg] = {-1, -1};
                    break;
            }
        }
    }
    // the pools are freed when this returns; wait for the work that reads them
    return hip_check(hipStreamSynchronize(s), "sync");
}

// Scratch of the observed-data mode for records of up to n = nt * nrec values.
struct ObsScratch {
    DevBuf pred, res, part;
    std::vector<double> host;
    wf_status ensure(int64_t n) {
        const int64_t nb = residual_blocks(std::max<int64_t>(n, 1));
        if (pred.bytes < n * 4) WF_TRY(pred.alloc(std::max<int64_t>(n, 1) * 4));
        if (res.bytes < n * 4) WF_TRY(res.alloc(std::max<int64_t>(n, 1) * 4));
        if (part.bytes < nb * 8) WF_TRY(part.alloc(nb * 8));
        return WF_OK;
    }
    int64_t bytes() const { return pred.bytes + res.bytes + part.bytes; }
    // 1/2 |r|^2 from the partial sums
    wf_status misfit(int64_t n, hipStream_t s, double* out) {
        *out = 0.0;
        if (n <= 0) return WF_OK;
        host.assign((size_t)residual_blocks(n), 0.0);
        WF_TRY(hip_check(hipMemcpyAsync(host.data(), part.ptr, host.size() * 8, hipMemcpyDeviceToHost, s),
                         "read misfit"));
        WF_TRY(hip_check(hipStreamSynchronize(s), "sync"));
        double phi = 0.0;
        for (double v : host) phi += v;   // fixed order: deterministic
        *out = 0.5 * phi;
        return WF_OK;
    }
};

}  // namespace

wf_status run_gradient(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                       const PointSet& rec, const float* residual, float* grad_out, int n_ck,
                       int64_t budget, hipStream_t s, const float* d_obs, float* d_pred_out,
                       double* misfit_out) {
    const Layout& L = md.L;
    FieldPool acc;
    WF_TRY(acc.alloc(L, 1, s));   // zeroed accumulator
    ObsScratch sc;
    ObsData obs;
    const int64_t n = (int64_t)nt * rec.npts;
    if (d_obs) {
        WF_TRY(sc.ensure(n));
        obs.d_obs = d_obs;
        obs.d_pred = d_pred_out ? d_pred_out : sc.pred.f();
        obs.resid = sc.res.f();
        obs.partial = sc.part.as<double>();
    }
    WF_TRY(gradient_core(md, dt, nt, src, src_wav, rec, residual, d_obs ? &obs : nullptr, acc.at(0),
                         acc.own.bytes + sc.bytes(), n_ck, budget, s));
    WF_TRY(hip_check(launch_unpitch(acc.at(0), grad_out, L.nx, L.ny, L.nz, L.sx, L.sy, s), "unpitch"));
    if (d_obs) {
        double phi = 0.0;
        WF_TRY(sc.misfit(n, s, &phi));
        if (misfit_out) *misfit_out = phi;
    }
    return hip_check(hipStreamSynchronize(s), "sync");
}

wf_status run_fwi_gradient(Model& md, double dt, int nt, const std::vector<FwiShot>& shots,
                           float* grad_out, double* misfit_out, int n_ck, int64_t budget,
                           hipStream_t s) {
    const Layout& L = md.L;
    FieldPool acc;
    WF_TRY(acc.alloc(L, 1, s));   // the sum over shots, zeroed once
    ObsScratch sc;
    int64_t nmax = 0;
    for (const FwiShot& sh : shots) nmax = std::max<int64_t>(nmax, (int64_t)nt * sh.nrec);
    WF_TRY(sc.ensure(nmax));
    double phi = 0.0;
    for (const FwiShot& sh : shots) {
        const PointSet *src = nullptr, *rec = nullptr;
        WF_TRY(md.points(sh.nsrc, sh.src_xyz, &src));
        WF_TRY(md.points(sh.nrec, sh.rec_xyz, &rec));
        ObsData obs;
        obs.d_obs = sh.d_obs;
        obs.d_pred = sh.d_pred ? sh.d_pred : sc.pred.f();
        obs.resid = sc.res.f();
        obs.partial = sc.part.as<double>();
        WF_TRY(gradient_core(md, dt, nt, *src, sh.src_wav, *rec, nullptr, &obs, acc.at(0),
                             acc.own.bytes + sc.bytes(), n_ck, budget, s));
        double ph = 0.0;
        WF_TRY(sc.misfit((int64_t)nt * sh.nrec, s, &ph));
        phi += ph;
    }
    WF_TRY(hip_check(launch_unpitch(acc.at(0), grad_out, L.nx, L.ny, L.nz, L.sx, L.sy, s), "unpitch"));
    if (misfit_out) *misfit_out = phi;
    return hip_check(hipStreamSynchronize(s), "sync");
}

// ---------------------------------------------------------------------------
// linearised (Born) modelling
// ---------------------------------------------------------------------------
// Background step n (kModeBornSource) writes u^{n+1} over u^{n-1} and the
// scattered source W = -dm (u^{n+1} - 2 u^n + u^{n-1}); the scattered step n
// (kModeVolumeSource) then advances du with W / dt^2 weighted like a point
// source (dt^2 / a). Receivers: d^n = P_r u^n and dd^n = P_r du^n, sampled
// inside the two launches.
wf_status run_born(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                   const float* dm, const PointSet& rec, float* drec_out, float* rec_out,
                   hipStream_t s) {
    const Layout& L = md.L;
    const int64_t nrec = rec.npts;
    WF_TRY(md.ensure_kap(dt, s));
    FieldPool f;
    WF_TRY(f.alloc(L, 4, s));   // zeroed: du^n, du^{n-1}, W, dm (pitched)
    float* dA = f.at(0);
    float* dB = f.at(1);
    float* W = f.at(2);
    float* DM = f.at(3);
    WF_TRY(hip_check(launch_pitch(dm, DM, L.nx, L.ny, L.nz, L.sx, L.sy, s), "pitch dm"));
    float* A = md.u(0);
    float* B = md.u(1);
    WF_TRY(hip_check(launch_fill(A, L.elems, 0.0f, s), "fill"));
    WF_TRY(hip_check(launch_fill(B, L.elems, 0.0f, s), "fill"));
    StepParams pu, pd;
    md.fill_step(pu, dt, kModeBornSource);
    md.fill_step(pd, dt, kModeVolumeSource);
    pd.vsrc = W;
    Injector inj;
    WF_TRY(inj.prepare(md, src, pu, src_wav, nt, md.d_inc[0], s));
    // the separate injection kernel subtracts ufwd * inc * idt2 from grad:
    // with idt2 = 1 that is the Born source's share of the injected value
    StepParams pw = pu;
    pw.idt2 = 1.0f;
    if (nt == 1 && nrec > 0) {
        WF_TRY(hip_check(launch_fill(drec_out, nrec, 0.0f, s), "fill"));
        if (rec_out) WF_TRY(hip_check(launch_fill(rec_out, nrec, 0.0f, s), "fill"));
    }
    for (int n = 0; n + 1 < nt; ++n) {
        inj.configure(pu, n);
        set_sampling(pu, &rec, (rec_out && nrec) ? rec_out + (int64_t)n * nrec : nullptr);
        WF_TRY(step(pu, md, A, B, B, kModeBornSource, W, DM, s));
        WF_TRY(inj.after(md, n, B, W, DM, pw, s));
        set_sampling(pd, &rec, nrec ? drec_out + (int64_t)n * nrec : nullptr);
        WF_TRY(step(pd, md, dA, dB, dB, kModeVolumeSource, nullptr, nullptr, s));
        std::swap(A, B);
        std::swap(dA, dB);
    }
    if (nt > 1) {
        WF_TRY(sample(rec, dA, drec_out + (int64_t)(nt - 1) * nrec, s));
        if (rec_out) WF_TRY(sample(rec, A, rec_out + (int64_t)(nt - 1) * nrec, s));
    }
    // the pool is freed when this returns
    return hip_check(hipStreamSynchronize(s), "sync");
}

// ---------------------------------------------------------------------------
// batched forward shots
// ---------------------------------------------------------------------------
wf_status batch_forward_begin(Model& md, double dt, int nt, const PointSet& src, const float* wav,
                              const PointSet& rec, float* rec_out, hipStream_t s, BatchFwd& b) {
    const Layout& L = md.L;
    WF_TRY(md.ensure_kap(dt, s));
    b = BatchFwd();
    b.md = &md;
    b.src = &src;
    b.rec = &rec;
    b.nt = nt;
    b.rec_out = rec_out;
    b.A = md.u(0);
    b.B = md.u(1);
    WF_TRY(hip_check(launch_fill(b.A, L.elems, 0.0f, s), "fill"));
    WF_TRY(hip_check(launch_fill(b.B, L.elems, 0.0f, s), "fill"));
    StepParams& p = b.p;
    md.fill_step(p, dt);
    // many grids share each launch, so a grid does not need to spread itself
    // over the whole device; the chunk length trades warm-up re-reads against
    // the sequential per-plane latency of each block (measured on a mixed
    // stream of orders 4/8/12: 8 planes best in 2D, 16 in 3D)
    int cx = std::min(L.nx, md.geom.ndim == 2 ? 8 : 16);
    if (const char* e = std::getenv("WAVEFD_BATCH_CX")) cx = std::max(1, std::min(L.nx, std::atoi(e)));
    step_plan(p, md.geom.ndim, md.half, kModePlain, cx, p.tile);
    Injector inj;
    WF_TRY(inj.prepare(md, src, p, wav, nt, md.d_inc[0], s));
    if (src.nnodes > 0 && !inj.fz) return fail(WF_E_STATE, "sources cannot be injected by the batched kernel");
    inj.configure(p, 0);
    b.inj_stride = inj.fz ? inj.fz->nnodes : 0;
    set_sampling(p, &rec, rec.npts ? rec_out : nullptr);
    b.nblk = (p.nblocks + 7) / 8 * 8;
    if (nt == 1 && rec.npts > 0) WF_TRY(hip_check(launch_fill(rec_out, rec.npts, 0.0f, s), "fill"));
    return WF_OK;
}

BatchJob batch_forward_job(const BatchFwd& b, int k_steps, int block_begin) {
    BatchJob j;
    j.p = b.p;
    j.buf0 = b.A;
    j.buf1 = b.B;
    j.inj_stride = b.inj_stride;
    j.smp_stride = b.rec ? b.rec->npts : 0;
    j.n0 = b.n;
    j.nsteps = std::max(0, std::min(k_steps, b.nt - 1 - b.n));
    j.block_begin = block_begin;
    j.nblk = b.nblk;
    return j;
}

void batch_forward_advance(BatchFwd& b, int steps) {
    b.n += steps;
    if (steps & 1) std::swap(b.A, b.B);
}

wf_status batch_forward_finish(BatchFwd& b, hipStream_t s) {
    if (b.nt > 1 && b.rec && b.rec->npts > 0)
        WF_TRY(sample(*b.rec, b.A, b.rec_out + (int64_t)(b.nt - 1) * b.rec->npts, s));
    return WF_OK;
}

}  // namespace wf
