// Internal host-side types of the propagator library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <initializer_list>
#include <vector>

#include "../../include/wavefd.h"
#include "kernels.h"

namespace wf {

wf_status fail(wf_status code, const char* fmt, ...);
const char* last_error();
void clear_error();
wf_status hip_check(hipError_t e, const char* what);

void fd_weights(int half, double* alpha);
double abs_weight_sum(int half);
wf_status check_geom(const wf_geom* g);
void comp_shape(const wf_geom* g, int64_t* nx, int64_t* ny, int64_t* nz);
double critical_dt(const wf_geom* g, double vmax);
std::vector<float> eta_profile(const wf_geom* g, int axis);

// Sub-allocator over one device allocation (the serving engine's HBM budget):
// first fit with coalescing, 256-byte granularity, thread-safe.
struct Arena;
Arena* arena_create(int64_t bytes);          // nullptr on failure (message set)
void arena_destroy(Arena* a);
void* arena_alloc(Arena* a, int64_t bytes);   // nullptr when it does not fit
void arena_free(Arena* a, void* p);
int64_t arena_used(const Arena* a);
int64_t arena_largest_free(Arena* a);
// While set on a thread, DevBuf allocations made by that thread come from the
// arena (and are returned to it when freed, from any thread). `s` is the
// stream that thread enqueues its work on: freeing such a buffer first waits
// for it, so that no queued kernel still uses memory the arena hands out again.
void set_thread_arena(Arena* a, hipStream_t s = nullptr);

// Caller-provided device memory handed out front to back (the static scratch
// of the no-allocation entry point): while set on a thread, DevBuf
// allocations made by that thread are carved from it and never freed on
// their own; a carve beyond `size` fails with WF_E_BUDGET.
struct ScratchRegion {
    char* base = nullptr;
    int64_t size = 0;
    int64_t used = 0;
};
void set_thread_scratch(ScratchRegion* r);
bool thread_scratch_active();
bool thread_arena_active();

// Pinned host memory for the small uploads of one thread: while set, a
// DevBuf::upload that fits copies its data here and queues an asynchronous
// copy on `stream` instead of a synchronous one. The caller synchronises
// `stream` before it resets `used`, frees the staging or uses the uploaded
// buffers on another stream.
struct PinnedStaging {
    char* base = nullptr;
    int64_t size = 0;
    int64_t used = 0;
    hipStream_t stream = nullptr;
};
void set_thread_staging(PinnedStaging* p);

// Owned device allocation.
struct DevBuf {
    void* ptr = nullptr;
    int64_t bytes = 0;
    Arena* arena = nullptr;
    bool external = false;         // carved from a ScratchRegion: nothing to free
    hipStream_t owner = nullptr;   // arena buffers: the stream to wait for before freeing
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void reset();
    wf_status alloc(int64_t nbytes);
    wf_status upload(const void* host, int64_t nbytes);   // synchronous (asynchronous through a thread's PinnedStaging)
    float* f() const { return static_cast<float*>(ptr); }
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// Several small host tables uploaded with one synchronous copy: `pack`
// receives them at 256-byte aligned offsets and each part's DevBuf becomes a
// view into it (nothing of its own to free; valid while `pack` is).
struct UploadPart {
    DevBuf* buf;
    const void* host;
    int64_t bytes;
};
wf_status upload_packed(DevBuf& pack, std::initializer_list<UploadPart> parts);

// Pitched field layout of a computational grid: element (x, y, z) at
// x*sx + y*sy + z with sy >= nz a multiple of 4 (pad entries stay zero).
struct Layout {
    int ndim = 3;
    int nx = 0, ny = 1, nz = 0;
    int64_t sx = 0, sy = 0;
    int64_t elems = 0;        // pitched size of planes 0..nx-1 in floats
    int64_t npoints = 0;      // nx*ny*nz
    int64_t ghost_off = 0;    // kGhostPlanes * sx: plane 0 within an allocation
    int64_t alloc_elems = 0;  // (nx + 2 kGhostPlanes) * sx
    void init(const wf_geom* g);
    int64_t field_bytes() const { return alloc_elems * 4 + 256; }
    // plane 0 of a field allocation
    float* field(void* alloc) const { return static_cast<float*>(alloc) + ghost_off; }
};

// Injection nodes of a point set arranged for the fused step kernel of one
// launch plan: entries (one per owning thread and plane, holding that
// thread's 4 z nodes) grouped by block, by thread and by x inside a block,
// plus everything the increment kernel needs per node slot in that order.
// Where a launch's threads sit: block b = (chunk * nty + ity) * ntz + itz
// covers the inner tile [ity ty, (ity + 1) ty) x [itz tz, (itz + 1) tz) and
// planes [chunk cx, min((chunk + 1) cx, nx)), each extended by ey rows, 4 ez4
// nodes and ex planes on either side (clipped to the grid); the node at row
// r and float4 column c of that region belongs to thread (r + oy) bz + c +
// oz4, which holds the 4 z nodes of its float4 column. A node inside several
// blocks' extended regions gets an entry in each.
struct InjGeom {
    int tz = 0, ty = 0, bz = 0, nt = 0;
    int ey = 0, ez4 = 0, ex = 0;
    int oy = 0, oz4 = 0;
    int ntz = 0, nty = 0, cx = 0, nchunks = 0, nblocks = 0;
    int cap = 0;                           // entries a block can stage
    int tag = 0;                           // distinguishes plans of different kernels
};
struct FusedInj {
    int64_t key[16] = {};                  // the InjGeom it was built for
    bool ok = false;                       // false: a block exceeds the LDS cap
    int nentries = 0;                      // (thread, plane) entries
    int nnodes = 0;                        // increment slots: 4 per entry
    DevBuf blk, thr, x;                    // block offsets, per-thread ranges, entry plane
    DevBuf off, eta, seg, pt, w;           // increment inputs per slot (empty slots: no terms)
};

// Sparse points of one acquisition: a gather table for sampling and a
// node-grouped table for deterministic injection.
struct PointSet {
    int npts = 0, K = 0, nnodes = 0;
    int64_t gen = 0;                            // unique id of this table (graph keys)
    DevBuf d_pack;                              // holds the tables below
    DevBuf d_off, d_w;                          // [npts*K]
    DevBuf d_noff, d_neta, d_seg, d_ept, d_ew;  // injection by node
    std::vector<int64_t> h_noff;                // host copies of the node tables
    std::vector<float> h_neta, h_ew;
    std::vector<int> h_seg, h_ept;
    mutable std::vector<FusedInj*> fused_cache;
    wf_status build(const wf_geom* g, const Layout& L, int npts, const double* xyz);
    // tables for the fused injection of launch plan p (nullptr on failure)
    wf_status fused(const Layout& L, const StepParams& p, const FusedInj** out) const;
    wf_status fused(const Layout& L, const InjGeom& g, const FusedInj** out) const;
    PointSet() = default;
    PointSet(const PointSet&) = delete;
    PointSet& operator=(const PointSet&) = delete;
    ~PointSet();
};

}  // namespace wf

// Signature of a captured time loop.
struct GraphKey {
    std::vector<int64_t> v;
    bool operator==(const GraphKey& o) const { return v == o.v; }
};

struct PCache {
    uint64_t key = 0;
    wf::PointSet* ps = nullptr;
    uint64_t tick = 0;
    std::vector<double> coords;
};

struct wf_model {
    virtual ~wf_model() = default;
};

struct Model : public wf_model {
    wf_geom geom{};
    int half = 0;
    wf::Layout L;
    double alpha[wf::kMaxHalf + 1]{};
    wf::DevBuf d_m, d_kap, d_u[2], d_eta_pack, d_etax, d_etay, d_etaz, d_scratch;
    wf::DevBuf d_u2[2];    // the two-update loop's second pair of fields (made on first use)
    wf::DevBuf d_inc[3];   // precomputed injection increments (grow-only, stream-ordered reuse)
    wf::DevBuf ws;         // gradient workspace (checkpoint pool + adjoint pair), kept between calls
    bool ws_clean = false; // every ghost plane in ws is zero
    float m_min = 0.f, m_max = 0.f;
    double kap_dt = -1.0;
    std::vector<PCache> pcache;
    uint64_t tick = 0;
    hipStream_t last_stream = nullptr;   // the stream of the most recent work
    hipEvent_t order_ev = nullptr;       // orders work on a new stream after the last one
    // make `s` the model's stream: work enqueued on it from now on starts
    // after everything enqueued on the previous one (no host wait)
    wf_status use_stream(hipStream_t s);
    // captured time loops (forward or adjoint), least recently used first out
    struct GraphEntry {
        GraphKey key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t tick = 0;
    };
    static constexpr size_t kMaxGraphs = 4;   // captured loops kept per model
    static constexpr size_t kMaxSeen = 8;     // signatures remembered for capture
    std::vector<GraphEntry> graphs;
    std::vector<GraphKey> seen;               // recent eager signatures, oldest first
    uint64_t graph_tick = 0;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int64_t graph_launches = 0;
    wf_status ensure_graph_stream();
    void drop_graphs();

    ~Model() override;
    wf_status init(const wf_geom* g, const float* m_dev, hipStream_t s);
    // init without the two wavefields (a caller that keeps them elsewhere)
    // and with the check of m left pending: its min, max and invalid count
    // land in host3 (pinned) when `s` passes the copy; finish_m(host3)
    // after that completes the init
    wf_status init_pending(const wf_geom* g, const float* m_dev, hipStream_t s, unsigned int* host3);
    wf_status finish_m(const unsigned int* host3);
    wf_status set_m(const float* m_dev, hipStream_t s);
    wf_status refresh_m(hipStream_t s);
    // the physical grid as a box [b0, b1) per layout axis (x, y, z; y = [0, 1) in 2D)
    void interior(int b0[3], int b1[3]) const;
    // the face slabs around that box that its stencil reads (boundary strips)
    wf::StripGeom strips() const;
    // m <- min(max(m - alpha grad, lo), hi); m_out (optional) receives it
    wf_status update(const float* grad, double alpha, double lo, double hi, float* m_out, hipStream_t s);
    // WF_E_NONFINITE (naming `what`) if any of the n device floats at x is
    // not finite; waits for the stream
    wf_status check_finite(const float* x, int64_t n, const char* what, hipStream_t s);
    wf_status ensure_kap(double dt, hipStream_t s);
    wf_status check_dt(double dt) const;
    double vmax() const;
    wf_status points(int npts, const double* xyz, const wf::PointSet** out);
    // plan a step launch; sample_points > 0 leaves room for that many fused samples
    void fill_step(wf::StepParams& p, double dt, int mode = wf::kModePlain) const;
    float* u(int i) const { return L.field(d_u[i].ptr); }
    // fields 2 and 3 of the two-update loop (allocated, ghost planes zeroed, on first use)
    wf_status ensure_u2(hipStream_t s);
    float* u2(int i) const { return L.field(d_u2[i].ptr); }
    float* kap() const { return L.field(d_kap.ptr); }
    int64_t bytes() const {
        return d_m.bytes + d_kap.bytes + d_u[0].bytes + d_u[1].bytes + d_u2[0].bytes + d_u2[1].bytes + d_eta_pack.bytes + d_scratch.bytes + d_inc[0].bytes + d_inc[1].bytes + d_inc[2].bytes + ws.bytes;
    }
};

namespace wf {

// Kernel timing: while enabled, launches of `kind` are bracketed by events.
bool profiling_active();
struct ProfScope {
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int kind, hipStream_t s);
    ~ProfScope();
};
// While run timing is on: one event before a time loop's first step launch
// and one after its last (finish(n) with the loop's n step launches).
struct RunSpan {
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    explicit RunSpan(hipStream_t s, int kind = WF_KERNEL_STEP_RUN);
    void finish(int64_t launches);
    ~RunSpan();
};
// Every step launch is counted per kernel mode (wf_profile_step_launches);
// mode kModeCount counts the two-update launches.
void count_step_launch(int mode);

// Time loops (propagate.cpp).
// Process-wide switch for capturing time loops as HIP graphs.
void set_graphs_enabled(bool on);
// Process-wide mode of two updates per launch in 3D forward loops: 0 off,
// 1 where measured faster (step2_preferred), 2 wherever compiled.
void set_two_step_mode(int mode);
// While positive on a thread, the time loops that thread enqueues keep at
// most about 2 x `steps` step launches queued ahead of the device (a host
// wait on an event every `steps` launches), so that work other streams
// submit meanwhile is not stuck behind a whole loop in a shared hardware
// queue. Loops are not captured as graphs then.
void set_thread_throttle(int steps);
// post-run checks that every output value is finite (process-wide switch,
// initially on when WAVEFD_VALIDATE=1)
bool validation_enabled();
void set_validation(bool on);
// inc_buf: the buffer of the per-step injection increments (default: the
// model's own, grown as needed)
wf_status run_forward(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                      const PointSet& rec, float* rec_out, float* u_save, int save_every,
                      hipStream_t s, DevBuf* inc_buf = nullptr);
// WAVEFD_NO_FUSED_INJECT set: sources go through the separate injection kernel
bool fused_injection_disabled();
wf_status run_adjoint(Model& md, double dt, int nt, const PointSet& rec, const float* rec_in,
                      const PointSet& src, float* src_out, hipStream_t s);
// Adjoint-state gradient (dense grad_out, overwritten). With d_obs (device
// [nt][nrec]) the residual is formed from the call's own forward sweep
// (residual ignored): d_pred_out (optional) receives P_r u and misfit_out
// 1/2 |P_r u - d_obs|^2.
wf_status run_gradient(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                       const PointSet& rec, const float* residual, float* grad_out, int n_ck,
                       int64_t budget, hipStream_t s, const float* d_obs = nullptr,
                       float* d_pred_out = nullptr, double* misfit_out = nullptr);

// Linearised modelling dd = J dm (dm dense); rec_out (optional) receives the
// background record.
wf_status run_born(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                   const float* dm, const PointSet& rec, float* drec_out, float* rec_out,
                   hipStream_t s);

// Observed-data terms of one gradient sweep (device buffers [nt][nrec]).
struct ObsData {
    const float* d_obs = nullptr;
    float* d_pred = nullptr;    // receives P_r u
    float* resid = nullptr;     // receives P_r u - d_obs
    double* partial = nullptr;  // residual_blocks(nt nrec) FP64 partial sums of resid^2
};

// One source experiment of a multi-shot gradient (host coordinates; the
// point tables are looked up shot by shot, so any number of shots fits the
// model's table cache).
struct FwiShot {
    int nsrc = 0;
    const double* src_xyz = nullptr;
    const float* src_wav = nullptr;
    int nrec = 0;
    const double* rec_xyz = nullptr;
    const float* d_obs = nullptr;
    float* d_pred = nullptr;    // optional
};
wf_status run_fwi_gradient(Model& md, double dt, int nt, const std::vector<FwiShot>& shots,
                           float* grad_out, double* misfit_out, int n_ck, int64_t budget,
                           hipStream_t s);

// Batched forward shots (serving engine): a grid advanced by k_step_batch
// launches shared with other grids. begin() prepares fields, coefficients,
// injection increments and the launch plan; job() describes the next k steps;
// advance() moves the state on; finish() writes the last record row.
struct BatchFwd {
    Model* md = nullptr;
    const PointSet* src = nullptr;
    const PointSet* rec = nullptr;
    StepParams p{};
    float* A = nullptr;    // u^n
    float* B = nullptr;    // u^{n-1}
    int n = 0, nt = 0;
    int64_t inj_stride = 0;
    float* rec_out = nullptr;
    int nblk = 0;          // blocks of one step (sampling + stencil, multiples of 8)
};
wf_status batch_forward_begin(Model& md, double dt, int nt, const PointSet& src, const float* wav,
                              const PointSet& rec, float* rec_out, hipStream_t s, BatchFwd& b);
BatchJob batch_forward_job(const BatchFwd& b, int k_steps, int block_begin);
void batch_forward_advance(BatchFwd& b, int steps);
wf_status batch_forward_finish(BatchFwd& b, hipStream_t s);

// Free device memory the current thread may allocate (its arena, if any).
int64_t device_free_bytes();

// Nonzero values (NaN included) in the ghost planes and row padding of the
// model's kappa and wavefield buffers and, while it is marked clean, of every
// field slot of its gradient workspace. Synchronous.
wf_status count_ghost_nonzero(const Model& md, int64_t* out);

// Revolve schedule (revolve.cpp).
int64_t revolve_cost(int64_t steps, int snaps);
struct RevolveAction {
    // ADVANCE: forward from state `at` to state `arg`; TAKESHOT: pin the current
    // state (x_at) in slot `arg`; RESTORE: make slot `arg` (x_at) current;
    // REVERSE: the adjoint of step `at` (needs x_at current); FREE: release slot.
    enum Kind { ADVANCE, TAKESHOT, RESTORE, REVERSE, FREE } kind;
    int64_t at;
    int64_t arg;
};
wf_status revolve_schedule(int64_t steps, int snaps, std::vector<RevolveAction>& out);

}  // namespace wf
