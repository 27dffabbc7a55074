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

wf_status step(StepParams& p, const Model& md, const float* cur, const float* old, float* out,
               bool img, float* grad, const float* ufwd, hipStream_t s) {
    p.cur = cur;
    p.old = old;
    p.out = out;
    p.grad = grad;
    p.ufwd = ufwd;
    ProfScope prof(WF_KERNEL_STEP, s);
    return hip_check(launch_step(p, md.geom.ndim, md.half, img, s), "stencil launch");
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

}  // namespace

wf_status run_forward(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                      const PointSet& rec, float* rec_out, float* u_save, int save_every,
                      hipStream_t s) {
    const Layout& L = md.L;
    WF_TRY(md.ensure_kap(dt, s));
    float* A = md.u(0);   // u^n
    float* B = md.u(1);   // u^{n-1}, overwritten by u^{n+1}
    WF_TRY(hip_check(launch_fill(A, L.elems, 0.0f, s), "fill"));
    WF_TRY(hip_check(launch_fill(B, L.elems, 0.0f, s), "fill"));
    if (rec.npts > 0) WF_TRY(hip_check(launch_fill(rec_out, rec.npts, 0.0f, s), "fill"));
    if (u_save) WF_TRY(hip_check(launch_fill(u_save, L.npoints, 0.0f, s), "fill"));
    StepParams p;
    md.fill_step(p, dt);
    for (int n = 0; n + 1 < nt; ++n) {
        WF_TRY(step(p, md, A, B, B, false, nullptr, nullptr, s));
        WF_TRY(inject(md, src, src_wav + (int64_t)n * src.npts, B, nullptr, nullptr, p, s));
        WF_TRY(sample(rec, B, rec_out + (int64_t)(n + 1) * rec.npts, s));
        if (u_save && (n + 1) % save_every == 0)
            WF_TRY(hip_check(launch_unpitch(B, u_save + (int64_t)((n + 1) / save_every) * L.npoints,
                                            L.nx, L.ny, L.nz, L.sx, L.sy, s), "save"));
        std::swap(A, B);
    }
    return WF_OK;
}

wf_status run_adjoint(Model& md, double dt, int nt, const PointSet& rec, const float* rec_in,
                      const PointSet& src, float* src_out, hipStream_t s) {
    const Layout& L = md.L;
    WF_TRY(md.ensure_kap(dt, s));
    float* A = md.u(0);   // v^{n+1}
    float* B = md.u(1);   // v^{n+2}, overwritten by v^n
    WF_TRY(hip_check(launch_fill(A, L.elems, 0.0f, s), "fill"));
    WF_TRY(hip_check(launch_fill(B, L.elems, 0.0f, s), "fill"));
    if (src.npts > 0)
        WF_TRY(hip_check(launch_fill(src_out + (int64_t)(nt - 1) * src.npts, src.npts, 0.0f, s), "fill"));
    StepParams p;
    md.fill_step(p, dt);
    for (int n = nt - 2; n >= 0; --n) {
        WF_TRY(step(p, md, A, B, B, false, nullptr, nullptr, s));
        WF_TRY(inject(md, rec, rec_in + (int64_t)(n + 1) * rec.npts, B, nullptr, nullptr, p, s));
        WF_TRY(sample(src, B, src_out + (int64_t)n * src.npts, s));
        std::swap(A, B);
    }
    return WF_OK;
}

// ---------------------------------------------------------------------------
// gradient
// ---------------------------------------------------------------------------
namespace {

// A pool of pitched field buffers (with zero ghost planes) carved from one
// allocation, zeroed once.
struct FieldPool {
    DevBuf mem;
    int64_t stride = 0;   // floats per buffer
    int64_t off = 0;      // plane 0 within a buffer
    int count = 0;
    wf_status alloc(const Layout& L, int n, hipStream_t s) {
        stride = (L.alloc_elems + 63) / 64 * 64;
        off = L.ghost_off;
        count = n;
        wf_status st = mem.alloc((int64_t)n * stride * 4 + 256);
        if (st != WF_OK) return st;
        return hip_check(launch_fill(mem.f(), mem.bytes / 4, 0.0f, s), "fill");
    }
    float* at(int i) const { return mem.f() + (int64_t)i * stride + off; }
};

}  // namespace

wf_status run_gradient(Model& md, double dt, int nt, const PointSet& src, const float* src_wav,
                       const PointSet& rec, const float* residual, float* grad_out, int n_ck,
                       int64_t budget, hipStream_t s) {
    const Layout& L = md.L;
    const int64_t fb = ((L.alloc_elems + 63) / 64 * 64) * 4;
    WF_TRY(md.ensure_kap(dt, s));
    StepParams p, pi;
    md.fill_step(p, dt);
    md.fill_step(pi, dt, true);
    const int64_t l = nt - 1;                     // adjoint steps n = 0..nt-2
    if (l <= 0) {
        return hip_check(launch_fill(grad_out, L.npoints, 0.0f, s), "fill");
    }
    // memory plan: adjoint pair + gradient accumulator (3 fields) plus either
    // every forward field (store-all: nt fields incl. one zero field) or a
    // revolve pool of 2 s + 3 fields
    size_t free_b = 0, total_b = 0;
    WF_TRY(hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo"));
    int64_t cap = (int64_t)free_b - ((int64_t)256 << 20);
    if (budget > 0) cap = std::min<int64_t>(cap, budget);
    const int64_t fixed = 3 * fb;
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
        return fail(WF_E_ARG, "n_checkpoints must be >= -1");
    }
    if (!store_all) snaps = (int)std::min<int64_t>(snaps, l);
    const int nbuf = store_all ? nt : 2 * snaps + 3;
    const int64_t need = fixed + (int64_t)nbuf * fb;
    if (need > cap) return fail(WF_E_BUDGET, "gradient needs %lld bytes, %lld available", (long long)need, (long long)cap);

    FieldPool adj;
    WF_TRY(adj.alloc(L, 3, s));
    float* V1 = adj.at(0);   // v^{n+1}
    float* V2 = adj.at(1);   // v^{n+2}, overwritten by v^n
    float* G = adj.at(2);    // gradient accumulator (pitched)
    FieldPool pool;
    WF_TRY(pool.alloc(L, nbuf, s));

    auto reverse_step = [&](int64_t n, const float* u_np1) -> wf_status {
        WF_TRY(step(pi, md, V1, V2, V2, true, G, u_np1, s));
        WF_TRY(inject(md, rec, residual + (n + 1) * rec.npts, V2, G, u_np1, p, s));
        std::swap(V1, V2);
        return WF_OK;
    };

    if (store_all) {
        // buffer 0 is zero and stands for both u^0 and u^{-1}; buffer j holds u^j
        for (int64_t n = 0; n + 1 < nt; ++n) {
            const float* cur = pool.at((int)n);
            const float* old = pool.at((int)std::max<int64_t>(n - 1, 0));
            float* out = pool.at((int)(n + 1));
            WF_TRY(step(p, md, cur, old, out, false, nullptr, nullptr, s));
            WF_TRY(inject(md, src, src_wav + n * src.npts, out, nullptr, nullptr, p, s));
        }
        for (int64_t n = nt - 2; n >= 0; --n) WF_TRY(reverse_step(n, pool.at((int)(n + 1))));
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
        WF_TRY(step(p, md, pool.at(0), pool.at(1), pool.at(1), false, nullptr, nullptr, s));
        WF_TRY(inject(md, src, src_wav, pool.at(1), nullptr, nullptr, p, s));
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
                        WF_TRY(step(p, md, pool.at(bn), pool.at(bo), pool.at(out), false, nullptr, nullptr, s));
                        WF_TRY(inject(md, src, src_wav + (i + 1) * src.npts, pool.at(out), nullptr, nullptr, p, s));
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
                    WF_TRY(reverse_step(a.at, pool.at(bn)));
                    break;
                case RevolveAction::FREE:
                    --pin[slot[(size_t)a.arg].first];
                    --pin[slot[(size_t)a.arg].second];
                    slot[(size_t)a.arg] = {-1, -1};
                    break;
            }
        }
    }
    WF_TRY(hip_check(launch_unpitch(G, grad_out, L.nx, L.ny, L.nz, L.sx, L.sy, s), "unpitch"));
    // the pools are freed when this returns; wait for the work that reads them
    return hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace wf
