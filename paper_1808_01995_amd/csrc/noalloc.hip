// wf_forward_noalloc: forward modelling on an existing model with no device
// allocation. The sparse-point tables of the call's sources and receivers,
// the fused injection tables and the per-step injection increments (the
// scratch of wf_forward's kernels, which wf_forward allocates and caches) are
// carved from one file-scope device array instead; everything else is the
// model's, allocated when it was created.
#include <mutex>

#include "runtime.h"

namespace {

constexpr int64_t kScratchBytes = (int64_t)32 << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends. In host code this name is
// only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device.
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
wf_status scratch_address(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return wf::fail(WF_E_HIP, "hipGetDevice failed");
    }
    if (dev < 0 || dev >= kMaxDevices) return wf::fail(WF_E_STATE, "device %d beyond the supported %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return wf::fail(WF_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return WF_OK;
}

// The calling thread's DevBuf allocations come from the region while alive.
struct ScratchScope {
    wf::ScratchRegion reg;
    ScratchScope(char* base, int64_t size) {
        reg.base = base;
        reg.size = size;
        reg.used = 0;
        wf::set_thread_scratch(&reg);
    }
    ~ScratchScope() { wf::set_thread_scratch(nullptr); }
};

}  // namespace

extern "C" wf_status wf_forward_noalloc(wf_model* model, double dt, int nt, int nsrc, const double* src_xyz,
                                        const float* src_wav, int nrec, const double* rec_xyz, float* rec_out,
                                        void* stream) {
    try {
        using namespace wf;
        if (!model) return fail(WF_E_ARG, "model is NULL");
        Model& md = *static_cast<Model*>(model);
        if (nt < 1) return fail(WF_E_ARG, "nt must be >= 1");
        wf_status st;
        if ((st = md.check_dt(dt)) != WF_OK) return st;
        if (nsrc < 0 || nrec < 0) return fail(WF_E_ARG, "negative point count");
        if ((nsrc > 0 && (!src_wav || !src_xyz)) || (nrec > 0 && (!rec_out || !rec_xyz)))
            return fail(WF_E_ARG, "missing source or receiver arrays");
        if ((int64_t)nt * nsrc > ((int64_t)1 << 40) || (int64_t)nt * nrec > ((int64_t)1 << 40))
            return fail(WF_E_ARG, "series too large");
        char* base = nullptr;
        if ((st = scratch_address(&base)) != WF_OK) return st;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        // earlier calls on this stream may still read the scratch
        if ((st = hip_check(hipStreamSynchronize(s), "sync")) != WF_OK) return st;
        ScratchScope scope(base, kScratchBytes);
        // every scratch carve happens here, before any work is queued: the
        // point tables, the fused injection tables of this launch plan and
        // the increments of every step
        PointSet ps_src, ps_rec;
        if ((st = ps_src.build(&md.geom, md.L, nsrc, src_xyz)) != WF_OK) return st;
        if ((st = ps_rec.build(&md.geom, md.L, nrec, rec_xyz)) != WF_OK) return st;
        StepParams p;
        md.fill_step(p, dt, kModePlain);
        DevBuf inc;
        if (ps_src.nnodes > 0 && !fused_injection_disabled()) {
            const FusedInj* fz = nullptr;
            if ((st = ps_src.fused(md.L, p, &fz)) != WF_OK) return st;
            if (fz->ok && (st = inc.alloc((int64_t)nt * fz->nnodes * 4)) != WF_OK) return st;
        }
        st = run_forward(md, dt, nt, ps_src, src_wav, ps_rec, rec_out, nullptr, 1, s, &inc);
        if (st == WF_OK && validation_enabled()) st = md.check_finite(rec_out, (int64_t)nt * nrec, "rec_out", s);
        return st;
    } catch (const std::bad_alloc&) {
        return wf::fail(WF_E_NOMEM, "host allocation failed");
    } catch (...) {
        return wf::fail(WF_E_STATE, "internal error");
    }
}
