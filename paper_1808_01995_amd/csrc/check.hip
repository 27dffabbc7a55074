// Validation of the zero region around every field. Outside the computational
// grid the wavefield is zero (Section "Boundary conditions": the zero
// Dirichlet condition beyond the damping layer); the library stores that
// outside as ghost planes before and after the x range and as row padding
// beyond nz, which the stencil reads and no kernel may write. A nonzero value
// there means an out-of-range write, and would also break the gradient
// workspace's reuse, which skips re-clearing ghost planes it knows are clean.
#include <algorithm>

#include "runtime.h"

namespace {

__global__ void k_ghost_count(const float* __restrict__ f, int64_t ghost_off, int64_t elems,
                              int64_t alloc_elems, int64_t sy, int nz, unsigned long long* count) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < alloc_elems;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i - ghost_off;
        const bool outside = k < 0 || k >= elems || (k % sy) >= nz;
        if (outside && f[i] != 0.0f) ++c;   // NaN counts as nonzero
    }
    if (c) atomicAdd(count, c);
}

}  // namespace

namespace wf {

wf_status count_ghost_nonzero(const Model& md, int64_t* out) {
    *out = 0;
    const Layout& L = md.L;
    std::vector<const float*> allocs = {md.d_kap.f(), md.d_u[0].f(), md.d_u[1].f()};
    for (const DevBuf& b : md.d_u2)
        if (b.ptr) allocs.push_back(b.f());
    // every field slot of the gradient workspace while it is marked clean
    if (md.ws_clean && md.ws.ptr) {
        const int64_t stride = (L.alloc_elems + 63) / 64 * 64;
        const int64_t slots = (md.ws.bytes / 4) / stride;
        for (int64_t i = 0; i < slots; ++i) allocs.push_back(md.ws.f() + i * stride);
    }
    wf_status st = hip_check(hipStreamSynchronize(md.last_stream), "sync");
    if (st != WF_OK) return st;
    DevBuf cnt;
    if ((st = cnt.alloc(8)) != WF_OK) return st;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(WF_E_HIP, "stream");
    st = hip_check(hipMemsetAsync(cnt.ptr, 0, 8, s), "clear");
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((L.alloc_elems + 255) / 256, 4096));
    for (const float* a : allocs) {
        if (st != WF_OK) break;
        hipLaunchKernelGGL(k_ghost_count, dim3(grid), dim3(256), 0, s, a, L.ghost_off, L.elems, L.alloc_elems,
                           L.sy, L.nz, cnt.as<unsigned long long>());
        st = hip_check(hipGetLastError(), "ghost count");
    }
    unsigned long long host = 0;
    if (st == WF_OK) st = hip_check(hipMemcpyAsync(&host, cnt.ptr, 8, hipMemcpyDeviceToHost, s), "read");
    if (st == WF_OK) st = hip_check(hipStreamSynchronize(s), "sync");
    (void)hipStreamDestroy(s);
    if (st == WF_OK) *out = (int64_t)host;
    return st;
}

}  // namespace wf
