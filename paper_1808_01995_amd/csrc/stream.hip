// Bandwidth reference for the roofline (Section "Performance", subsection
// "Roofline analysis": the kernels are bounded by a measured stream bandwidth
// of the machine, a STREAM-TRIAD figure there). Here the stream moves the
// step kernel's traffic per node (three float reads, one float write) with
// no stencil, halo or reuse: one float4 per thread, non-temporal loads and
// stores, blocks in address order, which is the fastest of the stream shapes
// measured on the MI355X (grid-stride loops over persistent blocks ran 25 %
// slower on multi-GB arrays).
#include "runtime.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream(const v4f* __restrict__ a, const v4f* __restrict__ b,
                                                const v4f* __restrict__ c, v4f* __restrict__ o,
                                                int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n4) return;
    const v4f x = __builtin_nontemporal_load(a + i);
    const v4f y = __builtin_nontemporal_load(b + i);
    const v4f z = __builtin_nontemporal_load(c + i);
    __builtin_nontemporal_store(2.0f * x - y + z, o + i);
}

}  // namespace

using namespace wf;

extern "C" wf_status wf_stream_bandwidth(int64_t n_floats, int reps, double* gbs_out) {
    try {
        if (!gbs_out) return fail(WF_E_ARG, "gbs_out is NULL");
        *gbs_out = 0.0;
        if (n_floats < 1024 || n_floats > ((int64_t)1 << 34)) return fail(WF_E_ARG, "n_floats out of range");
        if (reps < 1) return fail(WF_E_ARG, "reps must be >= 1");
        const int64_t n4 = (n_floats + 3) / 4;
        const int64_t grid = (n4 + 255) / 256;
        DevBuf buf[4];
        for (auto& d : buf) {
            const wf_status sa = d.alloc(n4 * 16);
            if (sa != WF_OK) return sa;
        }
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(WF_E_HIP, "stream");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        wf_status st = WF_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(WF_E_HIP, "events");
        for (int k = 0; k < 4 && st == WF_OK; ++k)
            st = hip_check(hipMemsetAsync(buf[k].ptr, 0, (size_t)(n4 * 16), s), "clear");
        auto pass = [&]() {
            hipLaunchKernelGGL(k_stream, dim3((unsigned)grid), dim3(256), 0, s, buf[0].as<v4f>(),
                               buf[1].as<v4f>(), buf[2].as<v4f>(), buf[3].as<v4f>(), n4);
            return hip_check(hipGetLastError(), "stream kernel");
        };
        if (st == WF_OK) st = pass();   // warm-up
        if (st == WF_OK) st = hip_check(hipEventRecord(e0, s), "event");
        for (int r = 0; r < reps && st == WF_OK; ++r) st = pass();
        if (st == WF_OK) st = hip_check(hipEventRecord(e1, s), "event");
        if (st == WF_OK) st = hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.0f;
        if (st == WF_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (st == WF_OK && ms > 0.0f) *gbs_out = 16.0 * (double)n4 * 4.0 * reps / (ms * 1e-3) / 1e9;
        (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(s);
        return st;
    } catch (...) {
        return fail(WF_E_NOMEM, "stream bandwidth failed");
    }
}
