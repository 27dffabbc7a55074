// Host runtime behind include/wavefd.h: models, sparse-point tables, the time
// loops of forward, adjoint and gradient, and the error plumbing of the C ABI.
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace wf {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

wf_status fail(wf_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char* last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// finite-difference weights (eq. fdSpace): centred second derivative of order
// k = 2M, alpha_j = 2 (-1)^{j+1} (M!)^2 / (j^2 (M-j)! (M+j)!), alpha_0 = -2 sum.
// Evaluated as a product of small ratios in long double.
// ---------------------------------------------------------------------------
void fd_weights(int half, double* alpha) {
    long double s = 0.0L;
    for (int j = 1; j <= half; ++j) {
        // (M!)^2 / ((M-j)! (M+j)!) = prod_{i=1}^{j} (M - j + i) / (M + i)
        long double r = 1.0L;
        for (int i = 1; i <= j; ++i) r *= (long double)(half - j + i) / (long double)(half + i);
        long double a = 2.0L * r / ((long double)j * (long double)j);
        if ((j & 1) == 0) a = -a;
        alpha[j] = (double)a;
        s += a;
    }
    alpha[0] = (double)(-2.0L * s);
}

double abs_weight_sum(int half) {
    double a[kMaxHalf + 1];
    fd_weights(half, a);
    double s = std::fabs(a[0]);
    for (int j = 1; j <= half; ++j) s += 2.0 * std::fabs(a[j]);
    return s;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
wf_status check_geom(const wf_geom* g) {
    if (!g) return fail(WF_E_ARG, "geometry is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(WF_E_ARG, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->space_order < 4 || g->space_order > 2 * kMaxHalf || (g->space_order & 1))
        return fail(WF_E_ARG, "space_order must be even in [4, %d] (got %d)", 2 * kMaxHalf,
                    g->space_order);
    if (g->nbl < 0 || g->nbl > 4096) return fail(WF_E_ARG, "nbl out of range (%d)", g->nbl);
    for (int a = 0; a < g->ndim; ++a) {
        if (g->n[a] < 2) return fail(WF_E_ARG, "n[%d] must be >= 2", a);
        if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a])) return fail(WF_E_ARG, "h[%d] must be > 0", a);
        if (!std::isfinite(g->origin[a])) return fail(WF_E_ARG, "origin[%d] not finite", a);
        if (g->n[a] + 2 * (int64_t)g->nbl > (int64_t)1 << 20) return fail(WF_E_ARG, "axis %d too long", a);
    }
    if (!(g->c_ref > 0.0) || !std::isfinite(g->c_ref)) return fail(WF_E_ARG, "c_ref must be > 0");
    if (g->R < 0.0 || g->R >= 1.0) return fail(WF_E_ARG, "R must be in [0, 1)");
    if (g->eta_power < 0 || g->eta_power > 4) return fail(WF_E_ARG, "eta_power must be in [0, 4]");
    // the pitched field must be addressable
    int64_t nx = g->n[0] + 2 * g->nbl, nz = g->n[g->ndim - 1] + 2 * g->nbl;
    int64_t ny = g->ndim == 3 ? g->n[1] + 2 * g->nbl : 1;
    if (nx * ny * (nz + 64) > ((int64_t)1 << 40)) return fail(WF_E_ARG, "grid too large");
    return WF_OK;
}

void comp_shape(const wf_geom* g, int64_t* nx, int64_t* ny, int64_t* nz) {
    *nx = g->n[0] + 2 * g->nbl;
    *ny = g->ndim == 3 ? g->n[1] + 2 * g->nbl : 1;
    *nz = g->n[g->ndim - 1] + 2 * g->nbl;
}

double critical_dt(const wf_geom* g, double vmax) {
    double inv = 0.0;
    for (int a = 0; a < g->ndim; ++a) inv += 1.0 / (g->h[a] * g->h[a]);
    return 2.0 / (vmax * std::sqrt(abs_weight_sum(g->space_order / 2) * inv));
}

// Per-axis damping profile on the computational grid (Section "Boundary
// conditions"): eta_a(c) = eta_max_a (d/nbl)^p, d = nodes outside the physical
// range [nbl, nbl + n - 1], eta_max_a = 3 ln(1/R) / (2 nbl h_a c_ref).
std::vector<float> eta_profile(const wf_geom* g, int axis) {
    const int64_t n = g->n[axis];
    const int nbl = g->nbl;
    const int64_t Nc = n + 2 * (int64_t)nbl;
    std::vector<float> e((size_t)Nc, 0.0f);
    if (nbl == 0) return e;
    const double R = g->R > 0.0 ? g->R : 1e-3;
    const int p = g->eta_power > 0 ? g->eta_power : 2;
    const double emax = 3.0 * std::log(1.0 / R) / (2.0 * nbl * g->h[axis] * g->c_ref);
    for (int64_t c = 0; c < Nc; ++c) {
        double d = 0.0;
        if (c < nbl) d = (double)(nbl - c);
        else if (c > nbl + n - 1) d = (double)(c - (nbl + n - 1));
        e[(size_t)c] = (float)(emax * std::pow(d / nbl, p));
    }
    return e;
}

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
static thread_local Arena* t_arena = nullptr;
static thread_local hipStream_t t_arena_stream = nullptr;
static thread_local ScratchRegion* t_scratch = nullptr;
static thread_local PinnedStaging* t_staging = nullptr;
void set_thread_scratch(ScratchRegion* r) { t_scratch = r; }
void set_thread_staging(PinnedStaging* p) { t_staging = p; }
bool thread_scratch_active() { return t_scratch != nullptr; }
bool thread_arena_active() { return t_arena != nullptr; }
void set_thread_arena(Arena* a, hipStream_t s) {
    t_arena = a;
    t_arena_stream = a ? s : nullptr;
}

int64_t device_free_bytes() {
    if (t_arena) return arena_largest_free(t_arena);
    size_t f = 0, t = 0;
    if (hipMemGetInfo(&f, &t) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return (int64_t)f - ((int64_t)256 << 20);   // headroom for the runtime
}

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
    if (ptr && !external) {
        if (arena) {
            // hipFree waits for the device; the arena does not, so wait for
            // the stream the buffer's work was queued on (a no-op when that
            // work is done, as on every successful path)
            if (owner) (void)hipStreamSynchronize(owner);
            arena_free(arena, ptr);
        } else {
            hipFree(ptr);
        }
    }
    ptr = nullptr;
    bytes = 0;
    arena = nullptr;
    owner = nullptr;
    external = false;
}
wf_status DevBuf::alloc(int64_t nbytes) {
    reset();
    if (nbytes <= 0) return WF_OK;
    if (t_scratch) {
        const int64_t off = (t_scratch->used + 255) / 256 * 256;
        if (off + nbytes > t_scratch->size)
            return fail(WF_E_BUDGET, "the call needs more than its %lld-byte device scratch (%lld bytes in use, "
                        "%lld more requested)", (long long)t_scratch->size, (long long)off, (long long)nbytes);
        ptr = t_scratch->base + off;
        bytes = nbytes;
        external = true;
        t_scratch->used = off + nbytes;
        return WF_OK;
    }
    if (t_arena) {
        void* q = arena_alloc(t_arena, nbytes);
        if (!q) return fail(WF_E_BUDGET, "device arena exhausted (%lld bytes requested)", (long long)nbytes);
        ptr = q;
        bytes = nbytes;
        arena = t_arena;
        owner = t_arena_stream;
        return WF_OK;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(WF_E_NOMEM, "hipMalloc(%lld bytes): %s", (long long)nbytes, hipGetErrorString(e));
    }
    ptr = p;
    bytes = nbytes;
    return WF_OK;
}
wf_status DevBuf::upload(const void* host, int64_t nbytes) {
    wf_status st = alloc(nbytes);
    if (st != WF_OK) return st;
    if (nbytes <= 0) return WF_OK;
    if (t_staging && t_staging->base) {
        const int64_t off = (t_staging->used + 255) / 256 * 256;
        if (off + nbytes <= t_staging->size) {
            std::memcpy(t_staging->base + off, host, (size_t)nbytes);
            t_staging->used = off + nbytes;
            return hip_check(hipMemcpyAsync(ptr, t_staging->base + off, (size_t)nbytes, hipMemcpyHostToDevice,
                                            t_staging->stream),
                             "staged upload");
        }
    }
    hipError_t e = hipMemcpy(ptr, host, (size_t)nbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(WF_E_HIP, "hipMemcpy H2D: %s", hipGetErrorString(e));
    return WF_OK;
}

wf_status upload_packed(DevBuf& pack, std::initializer_list<UploadPart> parts) {
    int64_t total = 0;
    for (const UploadPart& q : parts) total = (total + 255) / 256 * 256 + std::max<int64_t>(q.bytes, 0);
    std::vector<char> host((size_t)total);
    int64_t off = 0;
    for (const UploadPart& q : parts) {
        off = (off + 255) / 256 * 256;
        if (q.bytes > 0) std::memcpy(host.data() + off, q.host, (size_t)q.bytes);
        off += std::max<int64_t>(q.bytes, 0);
    }
    for (const UploadPart& q : parts) q.buf->reset();
    wf_status st = pack.upload(host.data(), total);
    if (st != WF_OK) return st;
    off = 0;
    for (const UploadPart& q : parts) {
        off = (off + 255) / 256 * 256;
        if (q.bytes > 0) {
            q.buf->ptr = static_cast<char*>(pack.ptr) + off;
            q.buf->bytes = q.bytes;
            q.buf->external = true;
        }
        off += std::max<int64_t>(q.bytes, 0);
    }
    return WF_OK;
}

wf_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return WF_OK;
    (void)hipGetLastError();
    return fail(WF_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// fields
// ---------------------------------------------------------------------------
void Layout::init(const wf_geom* g) {
    int64_t x, y, z;
    comp_shape(g, &x, &y, &z);
    ndim = g->ndim;
    nx = (int)x;
    ny = (int)y;
    nz = (int)z;
    // z rows padded to whole 128-byte cache lines: the vector loads need a
    // multiple of 4 floats, line-aligned rows and 128-float tiles keep every
    // tile row on whole lines (measured: ~7% less traffic than 64-byte rows)
    int align = 32;
    if (const char* s = std::getenv("WAVEFD_PITCH_ALIGN")) {
        int v = std::atoi(s);
        if (v >= 4 && v <= 256 && (v % 4) == 0) align = v;
    }
    sy = ((int64_t)nz + align - 1) / align * align;
    sx = sy * ny;
    elems = sx * nx;
    npoints = (int64_t)nx * ny * nz;
    ghost_off = (int64_t)kGhostPlanes * sx;
    alloc_elems = (int64_t)(nx + 2 * kGhostPlanes) * sx;
}

// ---------------------------------------------------------------------------
// sparse points (Section "Sparse point interpolation"): multilinear weights in
// the containing cell, computed in FP64 on the host.
// ---------------------------------------------------------------------------
wf_status build_points(const wf_geom* g, const Layout& L, int npts, const double* xyz,
                       std::vector<int64_t>& off, std::vector<float>& w,
                       std::vector<float>* eta_node) {
    const int D = g->ndim;
    const int K = 1 << D;
    off.assign((size_t)npts * K, 0);
    w.assign((size_t)npts * K, 0.0f);
    if (eta_node) eta_node->assign((size_t)npts * K, 0.0f);
    std::vector<std::vector<float>> prof;
    if (eta_node)
        for (int a = 0; a < D; ++a) prof.push_back(eta_profile(g, a));
    const int64_t Nc[3] = {L.nx, D == 3 ? L.ny : L.nz, L.nz};
    const int64_t stride[3] = {L.sx, D == 3 ? L.sy : 1, 1};
    for (int p = 0; p < npts; ++p) {
        int64_t base[3];
        double frac[3];
        for (int a = 0; a < D; ++a) {
            const double x = xyz[(size_t)p * D + a];
            if (!std::isfinite(x)) return fail(WF_E_DOMAIN, "point %d: coordinate not finite", p);
            const double s = (x - g->origin[a]) / g->h[a] + g->nbl;
            if (s < 0.0 || s > (double)(Nc[a] - 1))
                return fail(WF_E_DOMAIN, "point %d lies outside the computational grid on axis %d", p, a);
            int64_t i = (int64_t)std::floor(s);
            double f = s - (double)i;
            if (i >= Nc[a] - 1) {
                i = Nc[a] - 2;
                f = 1.0;
            }
            base[a] = i;
            frac[a] = f;
        }
        for (int k = 0; k < K; ++k) {
            int64_t o = 0;
            double wt = 1.0;
            float e = 0.0f;
            for (int a = 0; a < D; ++a) {
                const int bit = (k >> (D - 1 - a)) & 1;
                o += (base[a] + bit) * stride[a];
                wt *= bit ? frac[a] : 1.0 - frac[a];
                if (eta_node) e += prof[a][(size_t)(base[a] + bit)];
            }
            off[(size_t)p * K + k] = o;
            w[(size_t)p * K + k] = (float)wt;
            if (eta_node) (*eta_node)[(size_t)p * K + k] = e;
        }
    }
    return WF_OK;
}

#define WF_TRY_RT(expr)                      \
    do {                                     \
        wf_status st__ = (expr);             \
        if (st__ != WF_OK) return st__;      \
    } while (0)

static std::atomic<int64_t> g_pointset_gen{1};

wf_status PointSet::build(const wf_geom* g, const Layout& L, int npts_, const double* xyz) {
    gen = g_pointset_gen.fetch_add(1);
    npts = npts_;
    K = 1 << g->ndim;
    nnodes = 0;
    if (npts <= 0) return WF_OK;
    std::vector<int64_t> off;
    std::vector<float> w, e;
    wf_status st = build_points(g, L, npts, xyz, off, w, &e);
    if (st != WF_OK) return st;
    // sampling table: as is; injection table: entries grouped by node, in (point, corner) order inside
    // a node, so every node is summed by one thread in a fixed order
    const size_t ne = off.size();
    std::vector<size_t> idx(ne);
    for (size_t i = 0; i < ne; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return off[a] < off[b]; });
    std::vector<int64_t> noff;
    std::vector<float> neta, ew;
    std::vector<int> seg, ept;
    for (size_t t = 0; t < ne; ++t) {
        const size_t i = idx[t];
        if (t == 0 || off[i] != off[idx[t - 1]]) {
            seg.push_back((int)t);
            noff.push_back(off[i]);
            neta.push_back(e[i]);
        }
        ept.push_back((int)(i / K));
        ew.push_back(w[i]);
    }
    seg.push_back((int)ne);
    nnodes = (int)noff.size();
    st = upload_packed(d_pack, {{&d_off, off.data(), (int64_t)off.size() * 8},
                                {&d_w, w.data(), (int64_t)w.size() * 4},
                                {&d_noff, noff.data(), (int64_t)noff.size() * 8},
                                {&d_neta, neta.data(), (int64_t)neta.size() * 4},
                                {&d_seg, seg.data(), (int64_t)seg.size() * 4},
                                {&d_ept, ept.data(), (int64_t)ept.size() * 4},
                                {&d_ew, ew.data(), (int64_t)ew.size() * 4}});
    if (st != WF_OK) return st;
    h_noff = std::move(noff);
    h_neta = std::move(neta);
    h_seg = std::move(seg);
    h_ept = std::move(ept);
    h_ew = std::move(ew);
    return WF_OK;
}

PointSet::~PointSet() {
    for (FusedInj* f : fused_cache) delete f;
}

wf_status PointSet::fused(const Layout& L, const StepParams& p, const FusedInj** out) const {
    const TileShape ts = step_tile(L.ndim, p.tile);
    InjGeom g;
    g.tz = 4 * ts.bz;
    g.ty = ts.by;
    g.bz = ts.bz;
    g.nt = ts.bz * ts.by;
    g.ntz = p.ntz;
    g.nty = p.nty;
    g.cx = p.cx;
    g.nchunks = p.nchunks;
    g.nblocks = p.nblocks;
    g.cap = inj_cap(L.ndim);
    g.tag = p.tile;
    return fused(L, g, out);
}

wf_status PointSet::fused(const Layout& L, const InjGeom& g, const FusedInj** out) const {
    *out = nullptr;
    const int64_t key[16] = {g.tz, g.ty, g.bz, g.nt, g.ey, g.ez4, g.ex, g.oy, g.oz4, g.ntz, g.nty, g.cx,
                             g.nchunks, g.nblocks, g.cap, g.tag};
    for (FusedInj* f : fused_cache)
        if (std::equal(key, key + 16, f->key)) {
            *out = f;
            return WF_OK;
        }
    FusedInj* f = new (std::nothrow) FusedInj();
    if (!f) return fail(WF_E_NOMEM, "host allocation");
    std::copy(key, key + 16, f->key);
    const int NT = g.nt;
    // every (block, thread) whose extended region holds a node: the node's
    // plane and component
    struct Own { int64_t blk; int tid; int x; int comp; int node; };
    std::vector<Own> own;
    own.reserve((size_t)nnodes);
    const int ez = 4 * g.ez4;
    for (int k = 0; k < nnodes; ++k) {
        const int64_t o = h_noff[(size_t)k];
        const int x = (int)(o / L.sx);
        const int64_t rem = o % L.sx;
        const int y = (int)(rem / L.sy), z = (int)(rem % L.sy);
        const int ich0 = std::max(0, (x - g.ex) / g.cx - 1), ich1 = std::min(g.nchunks - 1, (x + g.ex) / g.cx + 1);
        const int ity0 = std::max(0, (y - g.ey) / g.ty - 1), ity1 = std::min(g.nty - 1, (y + g.ey) / g.ty + 1);
        const int itz0 = std::max(0, (z - ez) / g.tz - 1), itz1 = std::min(g.ntz - 1, (z + ez) / g.tz + 1);
        for (int ich = ich0; ich <= ich1; ++ich) {
            const int xb = ich * g.cx, xe = std::min(xb + g.cx, L.nx);
            if (x < xb - g.ex || x >= xe + g.ex) continue;
            for (int ity = ity0; ity <= ity1; ++ity) {
                const int yl = y - (ity * g.ty - g.ey);
                if (yl < 0 || yl >= g.ty + 2 * g.ey) continue;
                for (int itz = itz0; itz <= itz1; ++itz) {
                    const int zl = z - (itz * g.tz - ez);
                    if (zl < 0 || zl >= g.tz + 2 * ez) continue;
                    const int64_t b = ((int64_t)ich * g.nty + ity) * g.ntz + itz;
                    own.push_back({b, (yl + g.oy) * g.bz + zl / 4 + g.oz4, x, zl % 4, k});
                }
            }
        }
    }
    std::sort(own.begin(), own.end(), [](const Own& a, const Own& b) {
        if (a.blk != b.blk) return a.blk < b.blk;
        if (a.tid != b.tid) return a.tid < b.tid;
        if (a.x != b.x) return a.x < b.x;
        return a.comp < b.comp;
    });
    // entries: one per (block, thread, plane), 4 increment slots each (the
    // thread's 4 z nodes; an empty slot has no terms and so a zero increment)
    std::vector<int> blk((size_t)g.nblocks + 1, 0), xs, segs(1, 0), pts;
    std::vector<int2> thr((size_t)g.nblocks * NT, make_int2(0, 0));
    std::vector<int64_t> offs;
    std::vector<float> etas, ws;
    f->ok = true;
    size_t i = 0;
    int ne = 0;
    for (int64_t b = 0; b < g.nblocks; ++b) {
        blk[(size_t)b] = ne;
        const int e_b0 = ne;
        while (i < own.size() && own[i].blk == b) {
            const int t0 = ne;
            const int tid = own[i].tid;
            while (i < own.size() && own[i].blk == b && own[i].tid == tid) {
                const int x = own[i].x;
                int node_of[4] = {-1, -1, -1, -1};
                while (i < own.size() && own[i].blk == b && own[i].tid == tid && own[i].x == x) {
                    node_of[own[i].comp] = own[i].node;
                    ++i;
                }
                xs.push_back(x);
                for (int c = 0; c < 4; ++c) {
                    const int k = node_of[c];
                    if (k >= 0) {
                        offs.push_back(h_noff[(size_t)k]);
                        etas.push_back(h_neta[(size_t)k]);
                        for (int e = h_seg[(size_t)k]; e < h_seg[(size_t)k + 1]; ++e) {
                            pts.push_back(h_ept[(size_t)e]);
                            ws.push_back(h_ew[(size_t)e]);
                        }
                    } else {
                        offs.push_back(0);   // any valid node: its coefficient multiplies 0
                        etas.push_back(0.0f);
                    }
                    segs.push_back((int)pts.size());
                }
                ++ne;
            }
            thr[(size_t)(b * NT + tid)] = make_int2(t0, ne);
        }
        if (ne - e_b0 > g.cap) f->ok = false;
    }
    blk[(size_t)g.nblocks] = ne;
    f->nentries = ne;
    f->nnodes = 4 * ne;
    wf_status st;
    if (f->ok) {
        if ((st = f->blk.upload(blk.data(), (int64_t)blk.size() * 4)) != WF_OK ||
            (st = f->thr.upload(thr.data(), (int64_t)thr.size() * 8)) != WF_OK ||
            (st = f->x.upload(xs.data(), (int64_t)xs.size() * 4)) != WF_OK ||
            (st = f->off.upload(offs.data(), (int64_t)offs.size() * 8)) != WF_OK ||
            (st = f->eta.upload(etas.data(), (int64_t)etas.size() * 4)) != WF_OK ||
            (st = f->seg.upload(segs.data(), (int64_t)segs.size() * 4)) != WF_OK ||
            (st = f->pt.upload(pts.data(), (int64_t)pts.size() * 4)) != WF_OK ||
            (st = f->w.upload(ws.data(), (int64_t)ws.size() * 4)) != WF_OK) {
            delete f;
            return st;
        }
    }
    fused_cache.push_back(f);
    *out = f;
    return WF_OK;
}

uint64_t hash_points(int npts, int D, const double* xyz) {
    uint64_t h = 1469598103934665603ull ^ (uint64_t)npts ^ ((uint64_t)D << 40);
    const unsigned char* b = reinterpret_cast<const unsigned char*>(xyz);
    const size_t n = (size_t)npts * D * sizeof(double);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace wf

// ===========================================================================
// model
// ===========================================================================
using namespace wf;

wf_status Model::init(const wf_geom* g, const float* m_dev, hipStream_t s) {
    geom = *g;
    half = g->space_order / 2;
    L.init(g);
    fd_weights(half, alpha);
    wf_status st;
    const int64_t fb = L.field_bytes();
    if ((st = d_m.alloc(L.npoints * 4)) != WF_OK) return st;
    if ((st = d_kap.alloc(fb)) != WF_OK) return st;
    if ((st = d_u[0].alloc(fb)) != WF_OK) return st;
    if ((st = d_u[1].alloc(fb)) != WF_OK) return st;
    // ghost planes and pads must read as zero
    for (DevBuf* b : {&d_kap, &d_u[0], &d_u[1]})
        if ((st = hip_check(launch_fill(b->f(), b->bytes / 4, 0.0f, s), "fill")) != WF_OK) return st;
    std::vector<float> ex = eta_profile(g, 0);
    std::vector<float> ey = g->ndim == 3 ? eta_profile(g, 1) : std::vector<float>(1, 0.0f);
    std::vector<float> ez = eta_profile(g, g->ndim - 1);
    st = upload_packed(d_eta_pack, {{&d_etax, ex.data(), (int64_t)ex.size() * 4},
                                    {&d_etay, ey.data(), (int64_t)ey.size() * 4},
                                    {&d_etaz, ez.data(), (int64_t)ez.size() * 4}});
    if (st != WF_OK) return st;
    if ((st = d_scratch.alloc(256)) != WF_OK) return st;
    return set_m(m_dev, s);
}

wf_status Model::ensure_u2(hipStream_t s) {
    if (d_u2[0].ptr && d_u2[1].ptr) return WF_OK;
    const int64_t fb = L.field_bytes();
    wf_status st;
    for (DevBuf& b : d_u2) {
        if (b.ptr) continue;
        if ((st = b.alloc(fb)) != WF_OK) return st;
        // ghost planes and pads must read as zero
        if ((st = hip_check(launch_fill(b.f(), b.bytes / 4, 0.0f, s), "fill")) != WF_OK) return st;
    }
    return WF_OK;
}

wf_status Model::init_pending(const wf_geom* g, const float* m_dev, hipStream_t s, unsigned int* host3) {
    if (!m_dev) return fail(WF_E_ARG, "m is NULL");
    geom = *g;
    half = g->space_order / 2;
    L.init(g);
    fd_weights(half, alpha);
    WF_TRY_RT(d_m.alloc(L.npoints * 4));
    WF_TRY_RT(d_kap.alloc(L.field_bytes()));
    WF_TRY_RT(hip_check(launch_fill(d_kap.f(), d_kap.bytes / 4, 0.0f, s), "fill"));
    std::vector<float> ex = eta_profile(g, 0);
    std::vector<float> ey = g->ndim == 3 ? eta_profile(g, 1) : std::vector<float>(1, 0.0f);
    std::vector<float> ez = eta_profile(g, g->ndim - 1);
    WF_TRY_RT(upload_packed(d_eta_pack, {{&d_etax, ex.data(), (int64_t)ex.size() * 4},
                                         {&d_etay, ey.data(), (int64_t)ey.size() * 4},
                                         {&d_etaz, ez.data(), (int64_t)ez.size() * 4}}));
    WF_TRY_RT(d_scratch.alloc(256));
    WF_TRY_RT(use_stream(s));
    WF_TRY_RT(hip_check(hipMemcpyAsync(d_m.f(), m_dev, (size_t)L.npoints * 4, hipMemcpyDeviceToDevice, s), "copy m"));
    // min / max / invalid count of m, as refresh_m, read back without a wait
    float* d3 = d_scratch.f();
    WF_TRY_RT(hip_check(launch_fill(d3, 1, FLT_MAX, s), "init minmax"));
    WF_TRY_RT(hip_check(launch_fill(d3 + 1, 2, 0.0f, s), "init minmax"));
    WF_TRY_RT(hip_check(launch_minmax(d_m.f(), L.npoints, d3, s), "minmax"));
    WF_TRY_RT(hip_check(hipMemcpyAsync(host3, d3, 3 * sizeof(unsigned int), hipMemcpyDeviceToHost, s), "read minmax"));
    kap_dt = -1.0;
    return WF_OK;
}

wf_status Model::finish_m(const unsigned int* host3) {
    if (host3[2] != 0) return fail(WF_E_ARG, "m has %u values that are not positive and finite", host3[2]);
    std::memcpy(&m_min, &host3[0], 4);
    std::memcpy(&m_max, &host3[1], 4);
    return WF_OK;
}

wf_status Model::use_stream(hipStream_t s) {
    if (s == last_stream) return WF_OK;
    if (!order_ev)
        WF_TRY_RT(hip_check(hipEventCreateWithFlags(&order_ev, hipEventDisableTiming), "event"));
    WF_TRY_RT(hip_check(hipEventRecord(order_ev, last_stream), "record"));
    WF_TRY_RT(hip_check(hipStreamWaitEvent(s, order_ev, 0), "wait"));
    last_stream = s;
    return WF_OK;
}

wf_status Model::set_m(const float* m_dev, hipStream_t s) {
    if (!m_dev) return fail(WF_E_ARG, "m is NULL");
    WF_TRY_RT(use_stream(s));
    wf_status st;
    if ((st = hip_check(hipMemcpyAsync(d_m.f(), m_dev, (size_t)L.npoints * 4,
                                       hipMemcpyDeviceToDevice, s), "copy m")) != WF_OK)
        return st;
    return refresh_m(s);
}

// min / max of m (for the stability check) and validity of every value;
// invalidates the coefficients
wf_status Model::refresh_m(hipStream_t s) {
    wf_status st;
    unsigned int init3[3] = {0x7f7fffffu, 0u, 0u};
    unsigned int* d3 = reinterpret_cast<unsigned int*>(d_scratch.ptr);
    if ((st = hip_check(hipMemcpyAsync(d3, init3, sizeof init3, hipMemcpyHostToDevice, s), "init minmax")) != WF_OK)
        return st;
    if ((st = hip_check(launch_minmax(d_m.f(), L.npoints, reinterpret_cast<float*>(d3), s), "minmax")) != WF_OK)
        return st;
    unsigned int out3[3];
    if ((st = hip_check(hipMemcpyAsync(out3, d3, sizeof out3, hipMemcpyDeviceToHost, s), "read minmax")) != WF_OK)
        return st;
    if ((st = hip_check(hipStreamSynchronize(s), "sync")) != WF_OK) return st;
    if (out3[2] != 0) return fail(WF_E_ARG, "m has %u values that are not positive and finite", out3[2]);
    float lo, hi;
    std::memcpy(&lo, &out3[0], 4);
    std::memcpy(&hi, &out3[1], 4);
    m_min = lo;
    m_max = hi;
    kap_dt = -1.0;   // coefficients must be recomputed
    return WF_OK;
}

wf_status Model::check_finite(const float* x, int64_t n, const char* what, hipStream_t s) {
    if (!x || n <= 0) return WF_OK;
    unsigned int* cnt = reinterpret_cast<unsigned int*>(d_scratch.ptr);
    unsigned int bad = 0;
    WF_TRY_RT(hip_check(hipMemsetAsync(cnt, 0, 4, s), "clear"));
    WF_TRY_RT(hip_check(launch_count_nonfinite(x, n, cnt, s), "check finite"));
    WF_TRY_RT(hip_check(hipMemcpyAsync(&bad, cnt, 4, hipMemcpyDeviceToHost, s), "read"));
    WF_TRY_RT(hip_check(hipStreamSynchronize(s), "sync"));
    if (bad) return fail(WF_E_NONFINITE, "%s has %u values that are not finite", what, bad);
    return WF_OK;
}

namespace {
std::atomic<int>& validation_switch() {
    static std::atomic<int> on([] {
        const char* e = std::getenv("WAVEFD_VALIDATE");
        return (e && e[0] == '1') ? 1 : 0;
    }());
    return on;
}
}  // namespace

bool wf::validation_enabled() { return validation_switch().load(std::memory_order_relaxed) != 0; }
void wf::set_validation(bool on) { validation_switch().store(on ? 1 : 0); }

wf_status Model::update(const float* grad, double alpha, double lo, double hi, float* m_out,
                        hipStream_t s) {
    if (!grad) return fail(WF_E_ARG, "grad is NULL");
    if (!std::isfinite(alpha)) return fail(WF_E_ARG, "alpha must be finite");
    if (!(lo > 0.0) || !std::isfinite(lo) || !(hi >= lo))
        return fail(WF_E_ARG, "bounds must satisfy 0 < m_lo <= m_hi");
    const float flo = (float)lo;
    const float fhi = hi >= (double)FLT_MAX ? FLT_MAX : (float)hi;
    if (!(flo > 0.0f) || !(fhi >= flo)) return fail(WF_E_ARG, "bounds are not representable in FP32");
    WF_TRY_RT(use_stream(s));
    // a non-finite gradient value would be clamped silently: refuse it first
    WF_TRY_RT(check_finite(grad, L.npoints, "grad", s));
    WF_TRY_RT(hip_check(launch_update(d_m.f(), grad, (float)alpha, flo, fhi, L.npoints, s), "update"));
    if (m_out)
        WF_TRY_RT(hip_check(hipMemcpyAsync(m_out, d_m.f(), (size_t)L.npoints * 4, hipMemcpyDeviceToDevice, s),
                            "copy m"));
    return refresh_m(s);
}

void Model::interior(int b0[3], int b1[3]) const {
    const int nb = geom.nbl;
    b0[0] = nb;
    b1[0] = nb + (int)geom.n[0];
    if (geom.ndim == 3) {
        b0[1] = nb;
        b1[1] = nb + (int)geom.n[1];
    } else {
        b0[1] = 0;
        b1[1] = 1;
    }
    b0[2] = nb;
    b1[2] = nb + (int)geom.n[geom.ndim - 1];
}

StripGeom Model::strips() const {
    StripGeom g;
    g.sx = L.sx;
    g.sy = L.sy;
    int b0[3], b1[3];
    interior(b0, b1);
    const int N[3] = {L.nx, L.ny, L.nz};
    for (int a = 0; a < 3; ++a) {
        if (a == 1 && geom.ndim == 2) continue;
        for (int side = 0; side < 2; ++side) {
            int lo[3] = {b0[0], b0[1], b0[2]}, hi[3] = {b1[0], b1[1], b1[2]};
            if (side == 0) {
                lo[a] = std::max(0, b0[a] - half);
                hi[a] = b0[a];
            } else {
                lo[a] = b1[a];
                hi[a] = std::min(N[a], b1[a] + half);
            }
            if (hi[a] <= lo[a]) continue;
            const int k = g.nslab++;
            g.x0[k] = lo[0]; g.x1[k] = hi[0];
            g.y0[k] = lo[1]; g.y1[k] = hi[1];
            g.z0[k] = lo[2]; g.z1[k] = hi[2];
            g.start[k + 1] = g.start[k] + (int64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
        }
    }
    return g;
}

double Model::vmax() const { return 1.0 / std::sqrt(m_min); }

wf_status Model::ensure_kap(double dt, hipStream_t s) {
    WF_TRY_RT(use_stream(s));
    if (dt == kap_dt) return WF_OK;
    wf_status st = hip_check(launch_coef(d_m.f(), kap(), L.nx, L.ny, L.nz, L.sx, L.sy, dt, s), "coef");
    if (st != WF_OK) return st;
    kap_dt = dt;
    return WF_OK;
}

wf_status Model::check_dt(double dt) const {
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(WF_E_ARG, "dt must be > 0");
    const double dc = critical_dt(&geom, vmax());
    if (dt > dc * (1.0 + 1e-12))
        return fail(WF_E_CFL, "dt = %.6g ms exceeds the stability limit %.6g ms (vmax %.4g km/s)", dt, dc, vmax());
    return WF_OK;
}

wf_status Model::points(int npts, const double* xyz, const PointSet** out) {
    *out = nullptr;
    if (npts < 0) return fail(WF_E_ARG, "negative point count");
    if (npts > 0 && !xyz) return fail(WF_E_ARG, "coordinates are NULL");
    const uint64_t h = npts > 0 ? hash_points(npts, geom.ndim, xyz) : 0;
    for (auto& c : pcache)
        if (c.ps && c.key == h && c.ps->npts == npts && c.coords.size() == (size_t)npts * geom.ndim &&
            (npts == 0 || std::memcmp(c.coords.data(), xyz, c.coords.size() * sizeof(double)) == 0)) {
            c.tick = ++tick;
            *out = c.ps;
            return WF_OK;
        }
    PointSet* ps = new (std::nothrow) PointSet();
    if (!ps) return fail(WF_E_NOMEM, "host allocation");
    wf_status st = ps->build(&geom, L, npts, xyz);
    if (st != WF_OK) {
        delete ps;
        return st;
    }
    // evict the least recently used entry beyond the cache size (the device
    // work that may still read it is drained first)
    if (pcache.size() >= 16) {
        size_t lru = 0;
        for (size_t i = 1; i < pcache.size(); ++i)
            if (pcache[i].tick < pcache[lru].tick) lru = i;
        (void)hipStreamSynchronize(last_stream);
        delete pcache[lru].ps;
        pcache.erase(pcache.begin() + (long)lru);
    }
    PCache c;
    c.key = h;
    c.ps = ps;
    c.tick = ++tick;
    c.coords.assign(xyz, xyz + (size_t)npts * geom.ndim);
    pcache.push_back(std::move(c));
    *out = ps;
    return WF_OK;
}

wf_status Model::ensure_graph_stream() {
    if (gstream) return WF_OK;
    wf_status st = hip_check(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking), "stream");
    if (st == WF_OK) st = hip_check(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming), "event");
    if (st == WF_OK) st = hip_check(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming), "event");
    return st;
}

void Model::drop_graphs() {
    if (gstream) (void)hipStreamSynchronize(gstream);
    for (GraphEntry& e : graphs) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (e.graph) (void)hipGraphDestroy(e.graph);
    }
    graphs.clear();
    seen.clear();
}

Model::~Model() {
    (void)hipStreamSynchronize(last_stream);
    drop_graphs();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (order_ev) (void)hipEventDestroy(order_ev);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (auto& c : pcache) delete c.ps;
}

void Model::fill_step(StepParams& p, double dt, int mode) const {
    std::memset(&p, 0, sizeof p);
    p.kap = kap();
    p.etax = d_etax.f();
    p.etay = d_etay.f();
    p.etaz = d_etaz.f();
    p.nx = L.nx;
    p.ny = L.ny;
    p.nz = L.nz;
    p.sx = L.sx;
    p.sy = L.sy;
    double inv = 0.0;
    const double hx = geom.h[0], hz = geom.h[geom.ndim - 1];
    const double hy = geom.ndim == 3 ? geom.h[1] : 1.0;
    inv = 1.0 / (hx * hx) + 1.0 / (hz * hz) + (geom.ndim == 3 ? 1.0 / (hy * hy) : 0.0);
    p.c0 = (float)(alpha[0] * inv);
    for (int j = 1; j <= half; ++j) {
        p.wx[j] = (float)(alpha[j] / (hx * hx));
        p.wy[j] = geom.ndim == 3 ? (float)(alpha[j] / (hy * hy)) : 0.0f;
        p.wz[j] = (float)(alpha[j] / (hz * hz));
    }
    p.inv2dt = (float)(1.0 / (2.0 * dt));
    p.idt2 = (float)(1.0 / (dt * dt));
    // tuning overrides: WAVEFD_CX (x-chunk length), WAVEFD_TILE (3D tile shape 0/1)
    int cx = 0, tile = -1;
    if (const char* s = std::getenv("WAVEFD_CX")) cx = std::atoi(s);
    if (const char* s = std::getenv("WAVEFD_TILE")) tile = std::atoi(s);
    step_plan(p, geom.ndim, half, mode, cx, tile);
}
