// gfx950 kernels of the acoustic propagator.
//
// The hot kernel is the fused time update (eq. eulerfwd with the damping term
// of eq. fdWE-abc, centred in time):
//     out = (2 cur - (1 - g) old + kap * Lap(cur)) / (1 + g),
//     kap = dt^2 / m,  g = eta kap / (2 dt),
// where Lap is the sum over axes of the order-2M centred second difference
// (eq. fdSpace, centre weight once). It is bound by HBM bandwidth (about 2-4
// flop per byte against a ridge near 20), so it is organised around moving
// each byte once:
//   - blocks own a (y, z) tile and stream along x (the slowest axis);
//   - each thread holds 4 consecutive z points of one y row and keeps the
//     2M+1 x-neighbours of those points in registers, so x taps cost no
//     memory traffic;
//   - the current x-plane of the tile plus its y and z halos is staged in LDS
//     for the in-plane taps; halos are re-read from L2, not HBM, because
//     neighbouring tiles are scheduled on the same XCD at the same time;
//   - per point, HBM sees one read of cur, old and kap and one write of out
//     (16 bytes); the damping profile is three tiny per-axis tables.
#include "kernels.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <mutex>

namespace wf {

namespace {

__device__ __forceinline__ float4 ld4(const float* p) {
    return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ void st4(float* p, const float4& v) {
    *reinterpret_cast<float4*>(p) = v;
}
__device__ __forceinline__ float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// Streams that are read or written exactly once per step (the old field,
// kappa, the output) bypass L2 retention so that it keeps the current field,
// whose rows are re-read as halos by the neighbouring tiles.
#ifndef WF_STREAM_NT
#define WF_STREAM_NT 1
#endif
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4s(const float* p) {
#if WF_STREAM_NT
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
#else
    return *reinterpret_cast<const float4*>(p);
#endif
}
// The output store separately: WF_NT_OUT = 0 keeps the new field cacheable.
#ifndef WF_NT_OUT
#define WF_NT_OUT WF_STREAM_NT
#endif
// Planes of lookahead of the streamed operands and halos (1 or 2).
#ifndef WF_LA
#define WF_LA 1
#endif
__device__ __forceinline__ void st4o(float* p, const float4& v) {
#if WF_NT_OUT
    f4v t;
    t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
    __builtin_nontemporal_store(t, reinterpret_cast<f4v*>(p));
#else
    *reinterpret_cast<float4*>(p) = v;
#endif
}
__device__ __forceinline__ void st4s(float* p, const float4& v) {
#if WF_STREAM_NT
    f4v t;
    t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
    __builtin_nontemporal_store(t, reinterpret_cast<f4v*>(p));
#else
    *reinterpret_cast<float4*>(p) = v;
#endif
}
__device__ __forceinline__ float comp(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
__device__ __forceinline__ void set_comp(float4& v, int i, float s) {
    if (i == 0) v.x = s; else if (i == 1) v.y = s; else if (i == 2) v.z = s; else v.w = s;
}

// Block index -> tile index. Work-groups are dispatched to the 8 XCDs round
// robin; remapping makes each XCD own a contiguous run of tiles, so tiles that
// share halos share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = (nb + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// Planes of lookahead of the halo loads of the step kernel: M + PF (the
// distance at which the neighbouring blocks load the same rows into their
// rings) where the registers allow it, else the largest divisor of the ring
// length that keeps the kernel at its occupancy. WF_HL overrides it.
#ifndef WF_HL
#define WF_HL 0
#endif
__host__ __device__ constexpr int halo_lookahead(int M, int PF, bool d3, int mode) {
    const int nq = 2 * M + 1 + PF;
    // the imaging and source modes hold more operands per plane
    const bool plain = mode == 0;
    int cap = M + PF;
    if (d3 && plain && M > 4) cap = M <= 6 ? 2 : 3;
    if (d3 && !plain && M > 3) cap = M <= 6 ? 2 : 1;
    if (WF_HL > 0) cap = WF_HL;
    while (cap > 1 && nq % cap != 0) --cap;   // the largest divisor of the ring length up to cap
    return cap;
}

// One point's update, given its Laplacian.
__device__ __forceinline__ float update(float c, float old, float kap, float lap, float eta,
                                        float inv2dt) {
    const float g = eta * kap * inv2dt;
    const float num = fmaf(kap, lap, fmaf(g, old, 2.0f * c - old));
    return num * __builtin_amdgcn_rcpf(1.0f + g);
}

// ---------------------------------------------------------------------------
// Time step, 2D ([x][z]) or 3D ([x][y][z]).
//
// Block: BZ x BY threads over a (y, z) tile of TZ = 4 BZ by BY nodes; each
// thread owns 4 consecutive z nodes of one y row and walks its x range
// [xb, xe). The 2M+1 x-neighbours of the thread's column live in a ring of
// NQ = 2M + 1 + PF float4 registers; the x loop is unrolled by NQ so that the
// ring rotates by renaming (no register moves) and plane x + M + PF is loaded
// PF planes before it is first used. The old field, kappa and the y/z halos
// of the next plane are loaded one plane ahead. The staged plane alternates
// between two LDS buffers, so one barrier per plane suffices: a thread can
// only overwrite a buffer after every thread has passed the barrier of the
// plane in between.
// ---------------------------------------------------------------------------
template <bool D3, int M, int BZ, int BY, int PF, int MODE>
__device__ __forceinline__ void step_body(const StepParams& p, const int bidx) {
    constexpr bool IMG = MODE == kModeImaging;
    constexpr bool BSRC = MODE == kModeBornSource;
    constexpr bool VSRC = MODE == kModeVolumeSource;
    constexpr int NT = BZ * BY;
    constexpr int TZ = 4 * BZ;
    constexpr int P = (M + 3) & ~3;     // z halo rounded up to whole float4s
    constexpr int HZ = P / 4;
    constexpr int LW = TZ + 2 * P;      // LDS row (floats)
    constexpr int MY = D3 ? M : 0;      // y halo rows
    constexpr int LH = BY + 2 * MY;     // LDS rows per buffer
    constexpr int LBUF = LH * LW;
    constexpr int NQ = 2 * M + 1 + PF;
    constexpr int NHY = 2 * MY * BZ;    // y-halo float4 loads per plane
    constexpr int NHZ = 2 * BY * HZ;    // z-halo float4 loads per plane
    constexpr int JY = NHY > 0 ? (NHY + NT - 1) / NT : 1;
    constexpr int JZ = (NHZ + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) float lds[2 * LBUF];
    constexpr int ICAP = D3 ? kInjCap3 : kInjCap2;
    __shared__ int inj_xl[ICAP];
    __shared__ float4 inj_vl[ICAP];

    const int r = xcd_remap(bidx, p.nblocks);
    if (r >= p.nblocks) return;
    int t = r;
    const int itz = t % p.ntz;
    t /= p.ntz;
    const int ity = t % p.nty;
    const int ich = t / p.nty;

    const int tid = threadIdx.x;
    const int lz = tid % BZ, ly = tid / BZ;
    const int z0 = itz * TZ, y0 = ity * BY;
    const int z = z0 + 4 * lz, y = y0 + ly;
    const bool own = (y < p.ny) && (z < p.nz);
    const int xb = ich * p.cx;
    const int xe = min(xb + p.cx, p.nx);
    const int64_t sx = p.sx;
    // Loads are unconditional (a predicated load feeds a register merge that
    // would force the pipeline to drain): threads outside the grid read column
    // 0 and are masked where their values could reach a neighbour; x planes
    // beyond the grid are the zero ghost planes of the field allocation.
    const int64_t col = own ? (int64_t)y * p.sy + z : 0;

    // halo jobs of this thread (the same for every plane)
    int hy_l[JY], hz_l[JZ];
    int64_t hy_c[JY], hz_c[JZ];
    bool hy_v[JY], hz_v[JZ];
#pragma unroll
    for (int j = 0; j < JY; ++j) {
        const int i = tid + j * NT;
        hy_l[j] = -1;
        hy_v[j] = false;
        hy_c[j] = 0;
        if (i < NHY) {
            const int rr = i / BZ, cz = i - rr * BZ;
            const int lr = rr < MY ? rr : rr + BY;
            const int gy = y0 - MY + lr;
            const int gz = z0 + 4 * cz;
            hy_l[j] = lr * LW + P + 4 * cz;
            hy_v[j] = gy >= 0 && gy < p.ny && gz < p.nz;
            hy_c[j] = hy_v[j] ? (int64_t)gy * p.sy + gz : 0;
        }
    }
#pragma unroll
    for (int j = 0; j < JZ; ++j) {
        const int i = tid + j * NT;
        hz_l[j] = -1;
        hz_v[j] = false;
        hz_c[j] = 0;
        if (i < NHZ) {
            const int rr = i / (2 * HZ), k = i - rr * (2 * HZ);
            const int side = k / HZ, kk = k - side * HZ;
            const int lc = side ? (P + TZ + 4 * kk) : 4 * kk;
            const int gz = z0 - P + lc;
            const int gy = y0 + rr;
            hz_l[j] = (rr + MY) * LW + lc;
            hz_v[j] = gy < p.ny && gz >= 0 && gz < p.nz;
            hz_c[j] = hz_v[j] ? (int64_t)gy * p.sy + gz : 0;
        }
    }

    float eyz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        eyz[i] = (own && z + i < p.nz) ? ((D3 ? p.etay[y] : 0.0f) + p.etaz[z + i]) : 0.0f;

    // this block's injection nodes -> LDS (read only after the first barrier)
    int inj_i = 0, inj_e = 0, inj_nx = INT_MAX;
    float4 inj_nv = zero4();
    if (p.inj_blk) {
        const int b0 = p.inj_blk[r], b1 = p.inj_blk[r + 1];
        if (b1 > b0) {
            for (int i = tid; i < b1 - b0; i += NT) {
                inj_xl[i] = p.inj_x[b0 + i];
                inj_vl[i] = p.inj_inc[b0 + i];
            }
            const int2 rg = p.inj_thr[(int64_t)r * NT + tid];
            inj_i = rg.x - b0;
            inj_e = rg.y - b0;
            // the thread's next entry (plane and increments) lives in
            // registers: a plane without one costs one compare, and the LDS
            // reads of the following entry are not waited for in the plane
            // that issues them
            if (inj_i < inj_e) {
                inj_nx = p.inj_x[rg.x];
                inj_nv = p.inj_inc[rg.x];
            }
        }
    }

    float4 ring[NQ];
#pragma unroll
    for (int s = 0; s < 2 * M + PF; ++s) ring[s] = ld4(p.cur + (int64_t)(xb - M + s) * sx + col);
    ring[NQ - 1] = zero4();

    // old, kappa and the imaging/source operands of plane x are loaded LA
    // planes before x is computed, into register slot x % LA; the y/z halo
    // rows of plane x, HL planes before, into halo slot x % HL. With HL =
    // M + PF a block reads its neighbours' rows of a plane in the same
    // iteration as those neighbours load them into their own rings (blocks
    // sharing halos run side by side on one XCD), so the halo reads find the
    // rows in L2 rather than fetching them again from HBM. The ring length
    // NQ is a multiple of LA and HL, so every unrolled plane's slots are
    // compile-time constants.
    constexpr int LA = WF_LA;
    constexpr int HL = halo_lookahead(M, PF, D3, MODE);
    static_assert(NQ % LA == 0, "lookahead must divide the ring length");
    static_assert(NQ % HL == 0, "halo lookahead must divide the ring length");
    float4 uo_q[LA], kp_q[LA], uf_q[LA], gr_q[LA];
    float4 hy_q[HL][JY], hz_q[HL][JZ];
    float ex_q[LA];
    auto load_ahead = [&](int sl, int xx) {
        const int64_t b = (int64_t)xx * sx;
        ex_q[sl] = p.etax[min(xx, p.nx - 1)];
        uo_q[sl] = ld4s(p.old + b + col);
        kp_q[sl] = ld4s(p.kap + b + col);
        uf_q[sl] = zero4();
        gr_q[sl] = zero4();
        if (IMG) {
            uf_q[sl] = ld4s(p.ufwd + b + col);
            gr_q[sl] = ld4s(p.grad + b + col);
        }
        if (BSRC) uf_q[sl] = ld4s(p.ufwd + b + col);
        if (VSRC) uf_q[sl] = ld4s(p.vsrc + b + col);
    };
    auto load_halo = [&](int sl, int xx) {
        const int64_t b = (int64_t)xx * sx;
#pragma unroll
        for (int j = 0; j < JY; ++j) hy_q[sl][j] = ld4(p.cur + b + hy_c[j]);
#pragma unroll
        for (int j = 0; j < JZ; ++j) hz_q[sl][j] = ld4(p.cur + b + hz_c[j]);
    };
#pragma unroll
    for (int i = 0; i < HL; ++i) load_halo(i, xb + i);
#pragma unroll
    for (int i = 0; i < LA; ++i) load_ahead(i, xb + i);

    // this block's share of the receivers: interpolate cur (which the step
    // only reads); issued after the prologue loads so that the gather's
    // latency overlaps theirs. The corner order matches k_sample.
    if (p.smp_out) {
        constexpr int KS = D3 ? 8 : 4;   // corners of a cell
        const int s0 = r * p.smp_per, s1 = min(s0 + p.smp_per, p.smp_n);
        for (int i = s0 + tid; i < s1; i += NT) {
            int64_t so[KS];
            float sw[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                so[k] = p.smp_off[(int64_t)i * KS + k];
                sw[k] = p.smp_w[(int64_t)i * KS + k];
            }
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < KS; ++k) acc = fmaf(sw[k], p.cur[so[k]], acc);
            p.smp_out[i] = acc;
        }
    }

    for (int xg = xb; xg < xe; xg += NQ) {
#pragma unroll
        for (int ph = 0; ph < NQ; ++ph) {
            const int x = xg + ph;
            if (x < xe) {   // uniform; a guarded body keeps the loop fully unrollable
                // this plane's operands, loaded LA planes ago
                const int sl = ph % LA, hs = ph % HL;
                const float4 uo = uo_q[sl], kp = kp_q[sl], uf = uf_q[sl], gr = gr_q[sl];
                const float ex = ex_q[sl];
                float4 hy[JY], hz[JZ];
#pragma unroll
                for (int j = 0; j < JY; ++j) hy[j] = hy_q[hs][j];
#pragma unroll
                for (int j = 0; j < JZ; ++j) hz[j] = hz_q[hs][j];
                load_halo(hs, x + HL);    // planes from nx on are ghost planes
                load_ahead(sl, x + LA);
                ring[(ph + 2 * M + PF) % NQ] = ld4(p.cur + (int64_t)(x + M + PF) * sx + col);
                const float4 c = ring[(ph + M) % NQ];
                float* L = lds + (x & 1) * LBUF;
                float* lrow = L + (ly + MY) * LW;
                st4(lrow + P + 4 * lz, own ? c : zero4());
#pragma unroll
                for (int j = 0; j < JY; ++j)
                    if (hy_l[j] >= 0) st4(L + hy_l[j], hy_v[j] ? hy[j] : zero4());
#pragma unroll
                for (int j = 0; j < JZ; ++j)
                    if (hz_l[j] >= 0) st4(L + hz_l[j], hz_v[j] ? hz[j] : zero4());
                __syncthreads();

                float lap[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) lap[i] = p.c0 * comp(c, i);
#pragma unroll
                for (int j = 1; j <= M; ++j) {
                    const float4 a = ring[(ph + M - j) % NQ], b = ring[(ph + M + j) % NQ];
                    lap[0] = fmaf(p.wx[j], a.x + b.x, lap[0]);
                    lap[1] = fmaf(p.wx[j], a.y + b.y, lap[1]);
                    lap[2] = fmaf(p.wx[j], a.z + b.z, lap[2]);
                    lap[3] = fmaf(p.wx[j], a.w + b.w, lap[3]);
                }
                if (D3) {
#pragma unroll
                    for (int j = 1; j <= MY; ++j) {
                        const float4 a = ld4(lrow - j * LW + P + 4 * lz);
                        const float4 b = ld4(lrow + j * LW + P + 4 * lz);
                        lap[0] = fmaf(p.wy[j], a.x + b.x, lap[0]);
                        lap[1] = fmaf(p.wy[j], a.y + b.y, lap[1]);
                        lap[2] = fmaf(p.wy[j], a.z + b.z, lap[2]);
                        lap[3] = fmaf(p.wy[j], a.w + b.w, lap[3]);
                    }
                }
                {
                    float w[2 * P + 4];
#pragma unroll
                    for (int k = 0; k < (2 * P + 4) / 4; ++k) {
                        const float4 v = ld4(lrow + 4 * lz + 4 * k);
                        w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 1; j <= M; ++j)
                            lap[i] = fmaf(p.wz[j], w[P + i - j] + w[P + i + j], lap[i]);
                }

                if (VSRC) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) lap[i] = fmaf(comp(uf, i), p.idt2, lap[i]);
                }
                float4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = update(comp(c, i), comp(uo, i), comp(kp, i), lap[i], ex + eyz[i], p.inv2dt);
                    if (z + i >= p.nz) v = 0.0f;
                    set_comp(o, i, v);
                }
                float4 g2 = zero4();
                if (IMG) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float lapt = comp(o, i) - 2.0f * comp(c, i) + comp(uo, i);
                        set_comp(g2, i, comp(gr, i) - comp(uf, i) * lapt * p.idt2);
                    }
                }
                if (BSRC) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float lapt = comp(o, i) - 2.0f * comp(c, i) + comp(uo, i);
                        set_comp(g2, i, -comp(uf, i) * lapt);
                    }
                }
                // the source entry owned by this thread at this plane (rare,
                // divergent; nodes without a source have a zero increment)
                if (inj_nx == x) {
                    const float4 inc = inj_nv;
                    o.x += inc.x; o.y += inc.y; o.z += inc.z; o.w += inc.w;
                    if (IMG) {
                        g2.x -= uf.x * inc.x * p.idt2;
                        g2.y -= uf.y * inc.y * p.idt2;
                        g2.z -= uf.z * inc.z * p.idt2;
                        g2.w -= uf.w * inc.w * p.idt2;
                    }
                    if (BSRC) {
                        g2.x -= uf.x * inc.x;
                        g2.y -= uf.y * inc.y;
                        g2.z -= uf.z * inc.z;
                        g2.w -= uf.w * inc.w;
                    }
                    ++inj_i;
                    if (inj_i < inj_e) {
                        inj_nx = inj_xl[inj_i];
                        inj_nv = inj_vl[inj_i];
                    } else {
                        inj_nx = INT_MAX;
                    }
                }
                if (own) {
                    const int64_t base = (int64_t)x * sx;
                    st4o(p.out + base + col, o);
                    if (IMG || BSRC) st4s(p.grad + base + col, g2);
                }
            }
        }
    }
}

// Orders up to 8 in 3D keep at least 3 waves per SIMD (12 per CU, the
// residency the chunk planner assumes; VGPRs capped at 168). Higher orders
// would spill under that cap and run at 2.
template <bool D3, int M, int BZ, int BY, int PF, int MODE>
__global__ void __launch_bounds__(BZ * BY, (D3 && M <= 4) ? 3 : 1) k_step(const StepParams p) {
    step_body<D3, M, BZ, BY, PF, MODE>(p, (int)blockIdx.x);
}

// Many grids of one dimension and order advanced by one step in one launch
// (the serving engine's batch of small requests). Job j owns the blocks
// [block_begin, block_begin + nblk), block_begin a multiple of 8 so that each
// job's blocks keep their XCD placement; at launch step k the job advances from
// its step n0 + k, alternating its two fields, with this step's injection and
// sampling rows.
template <bool D3, int M, int BZ, int BY, int PF>
__global__ void __launch_bounds__(BZ * BY, (D3 && M <= 4) ? 3 : 1) k_step_batch(const BatchJob* __restrict__ jobs, int njobs,
                                                        int k) {
    int lo = 0, hi = njobs - 1;
    const int b = (int)blockIdx.x;
    while (lo < hi) {   // uniform binary search for the owning job
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const BatchJob& J = jobs[lo];
    if (k >= J.nsteps || b >= J.block_begin + J.nblk) return;
    StepParams p = J.p;
    const int64_t n = (int64_t)J.n0 + k;
    if (k & 1) {
        p.cur = J.buf1;
        p.old = J.buf0;
        p.out = J.buf0;
    } else {
        p.cur = J.buf0;
        p.old = J.buf1;
        p.out = J.buf1;
    }
    if (p.inj_blk) p.inj_inc += n * (J.inj_stride / 4);
    if (p.smp_out) p.smp_out += n * J.smp_stride;
    step_body<D3, M, BZ, BY, PF, kModePlain>(p, b - J.block_begin);
}

// ---------------------------------------------------------------------------
// Two plain updates per pass (2D and 3D): temporal blocking over overlapping
// tiles.
//
// Block: EY = BY + 2M rows (3D; one row in 2D) of BZE threads, one float4
// column each, over the extended tile; the inner tile is rows [M, M + BY)
// (3D) and columns [HZ, BZE - HZ). For its chunk [xb, xe) the block walks
// planes x = xb - M .. xe + M - 1: every thread forms u^{n+1}(x) of its
// column from a register ring of u^n planes (x taps) and an LDS plane of u^n
// that holds the extended tile plus a frame of M rows (3D) and P nodes (y and
// z taps), and
// keeps it in a register ring of u^{n+1} planes; the inner threads then form
// u^{n+2}(x - M) from that ring and an LDS plane of u^{n+1}(x - M), whose y
// and z neighbours the extended tile holds. u^{n+1} is zero outside the grid
// (columns outside it, planes outside [0, nx)), as the fields of the
// single-update loop are. Every node gets the arithmetic of step_body in the
// same order, so both fields equal two single updates bit for bit. Both LDS
// planes alternate between two buffers: one barrier per plane.
// ---------------------------------------------------------------------------
// PF: planes the u^n ring prefetches; LA: planes of lookahead of u^{n-1} and
// kap; KR: the second update reloads kap (else a register ring keeps M + 1
// planes of it, LA = 1 only); NTS: u^{n-1} and kap streamed non-temporal
// (else cached, so that the overlapping rows of neighbouring blocks can hit).
template <bool D3, int M, int BY, int BZE, int PF, int LA, bool KR, bool NTS>
__device__ __forceinline__ void step2_body(const Step2Params& p, const int bidx) {
    constexpr int HZ = (M + 3) / 4;
    constexpr int P = 4 * HZ;              // z extension and z frame (nodes)
    constexpr int TZ = 4 * (BZE - 2 * HZ); // inner tile along z
    constexpr int MY = D3 ? M : 0;         // y extension and y frame (rows)
    constexpr int EY = BY + 2 * MY;        // rows of the extended tile
    constexpr int NT = EY * BZE;
    constexpr int LWA = 4 * BZE + 2 * P;   // u^n plane: row width with the z frame
    constexpr int LBA = (EY + 2 * MY) * LWA;
    constexpr int LWU = 4 * BZE;           // u^{n+1} plane: the extended tile
    constexpr int LBU = EY * LWU;
    constexpr int NQ = 2 * M + 1 + PF;     // u^n ring; the u^{n+1} ring has the same length
    constexpr int KQ = KR ? 1 : M + 1;     // kap of planes x - M .. x
    constexpr int HL = 2;                  // planes of lookahead of the frame loads
    static_assert(NQ % KQ == 0 && NQ % HL == 0 && NQ % LA == 0, "ring lengths must divide the unrolled loop");
    static_assert(KR || LA == 1, "the kap ring takes the next plane only");
    // planes read beyond the chunk: u^n from xb - 2M to xe + 2M + PF - 1,
    // u^{n-1} and kap from xb - 2M to xe + M + LA - 1: all within the ghost planes
    static_assert(2 * M + PF <= kGhostPlanes && M + LA <= kGhostPlanes, "reads beyond the ghost planes");
    auto lds_ = [](const float* q) { return NTS ? ld4s(q) : ld4(q); };
    constexpr int NFY = 2 * MY * BZE;      // frame rows above and below (float4 loads)
    constexpr int NFZ = 2 * EY * HZ;       // frame columns left and right
    constexpr int JF = (NFY + NFZ + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) float la[2 * LBA];
    __shared__ __attribute__((aligned(16))) float lu[2 * LBU];
    constexpr int ICAP = step2_inj_cap(D3);
    __shared__ int inj_xl[2][ICAP];
    __shared__ float4 inj_vl[2][ICAP];

    const int r = xcd_remap(bidx, p.nblocks);
    if (r >= p.nblocks) return;
    int t = r;
    const int itz = t % p.ntz;
    t /= p.ntz;
    const int ity = t % p.nty;
    const int ich = t / p.nty;

    const int tid = threadIdx.x;
    const int lz = tid % BZE, ly = tid / BZE;
    const int z0 = itz * TZ, y0 = ity * BY;
    const int y = y0 - MY + ly, z = z0 - P + 4 * lz;
    const bool ing = y >= 0 && y < p.ny && z >= 0 && z < p.nz;
    const bool inner = ly >= MY && ly < MY + BY && lz >= HZ && lz < BZE - HZ;
    const int xb = ich * p.cx;
    const int xe = min(xb + p.cx, p.nx);
    const int xs = xb - M, xend = xe + M;
    const int64_t sx = p.sx;
    // as in step_body: unconditional loads, column 0 for threads outside the grid
    const int64_t col = ing ? (int64_t)y * p.sy + z : 0;

    int hf_l[JF];
    int64_t hf_c[JF];
    bool hf_v[JF];
#pragma unroll
    for (int j = 0; j < JF; ++j) {
        const int i = tid + j * NT;
        hf_l[j] = -1;
        hf_v[j] = false;
        hf_c[j] = 0;
        int gy = -1, gz = -1, l = -1;
        if (i < NFY) {
            const int rr = i / BZE, cz = i - rr * BZE;
            const int lr = rr < MY ? rr : rr + EY;
            gy = y0 - 2 * MY + lr;
            gz = z0 - P + 4 * cz;
            l = lr * LWA + P + 4 * cz;
        } else if (i < NFY + NFZ) {
            const int k = i - NFY;
            const int rr = k / (2 * HZ), kk = k - rr * (2 * HZ);
            const int side = kk / HZ, q = kk - side * HZ;
            const int lc = side ? (P + 4 * BZE + 4 * q) : 4 * q;
            gy = y0 - MY + rr;
            gz = z0 - 2 * P + lc;
            l = (rr + MY) * LWA + lc;
        }
        if (l >= 0) {
            hf_l[j] = l;
            hf_v[j] = gy >= 0 && gy < p.ny && gz >= 0 && gz < p.nz;
            hf_c[j] = hf_v[j] ? (int64_t)gy * p.sy + gz : 0;
        }
    }

    float eyz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        eyz[i] = (ing && z + i < p.nz) ? ((D3 ? p.etay[y] : 0.0f) + p.etaz[z + i]) : 0.0f;

    // injection entries of both updates -> LDS; each thread's next entry of
    // each list in registers (as in step_body)
    int inj_i[2] = {0, 0}, inj_e[2] = {0, 0}, inj_nx[2] = {INT_MAX, INT_MAX};
    float4 inj_nv[2] = {zero4(), zero4()};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!p.inj_blk[k]) continue;
        const int b0 = p.inj_blk[k][r], b1 = p.inj_blk[k][r + 1];
        if (b1 <= b0) continue;
        for (int i = tid; i < b1 - b0; i += NT) {
            inj_xl[k][i] = p.inj_x[k][b0 + i];
            inj_vl[k][i] = p.inj_inc[k][b0 + i];
        }
        const int2 rg = p.inj_thr[k][(int64_t)r * NT + tid];
        inj_i[k] = rg.x - b0;
        inj_e[k] = rg.y - b0;
        if (inj_i[k] < inj_e[k]) {
            inj_nx[k] = p.inj_x[k][rg.x];
            inj_nv[k] = p.inj_inc[k][rg.x];
        }
    }

    float4 ring[NQ], uring[NQ], kring[KQ], uo_q[LA], kp_q[LA];
#pragma unroll
    for (int s = 0; s < 2 * M + PF; ++s) ring[s] = ld4(p.cur + (int64_t)(xs - M + s) * sx + col);
    ring[NQ - 1] = zero4();
#pragma unroll
    for (int s = 0; s < NQ; ++s) uring[s] = zero4();
#pragma unroll
    for (int s = 0; s < KQ; ++s) kring[s] = zero4();
#pragma unroll
    for (int s = 0; s < LA; ++s) {
        uo_q[s] = lds_(p.old + (int64_t)(xs + s) * sx + col);
        kp_q[s] = KR ? lds_(p.kap + (int64_t)(xs + s) * sx + col) : zero4();
    }
    if (!KR) kring[0] = lds_(p.kap + (int64_t)xs * sx + col);
    float4 hq[HL][JF];
    auto load_frame = [&](int sl, int xx) {
        const int64_t b = (int64_t)xx * sx;
#pragma unroll
        for (int j = 0; j < JF; ++j) hq[sl][j] = ld4(p.cur + b + hf_c[j]);
    };
#pragma unroll
    for (int i = 0; i < HL; ++i) load_frame(i, xs + i);

    // this block's share of the receivers, from both fields it only reads
    // (k_sample's corner order)
    if (p.smp_cur || p.smp_old) {
        constexpr int KS = D3 ? 8 : 4;   // corners of a cell
        const int s0 = r * p.smp_per, s1 = min(s0 + p.smp_per, p.smp_n);
        for (int i = s0 + tid; i < s1; i += NT) {
            int64_t so[KS];
            float sw[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                so[k] = p.smp_off[(int64_t)i * KS + k];
                sw[k] = p.smp_w[(int64_t)i * KS + k];
            }
            if (p.smp_cur) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < KS; ++k) acc = fmaf(sw[k], p.cur[so[k]], acc);
                p.smp_cur[i] = acc;
            }
            if (p.smp_old) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < KS; ++k) acc = fmaf(sw[k], p.old[so[k]], acc);
                p.smp_old[i] = acc;
            }
        }
    }

    for (int xg = xs; xg < xend; xg += NQ) {
#pragma unroll
        for (int ph = 0; ph < NQ; ++ph) {
            const int x = xg + ph;
            if (x < xend) {   // uniform
                const float4 uo = uo_q[ph % LA];
                const float4 kp = KR ? kp_q[ph % LA] : kring[ph % KQ];
                float4 hf[JF];
#pragma unroll
                for (int j = 0; j < JF; ++j) hf[j] = hq[ph % HL][j];
                load_frame(ph % HL, x + HL);   // planes beyond the grid are ghost planes
                uo_q[ph % LA] = lds_(p.old + (int64_t)(x + LA) * sx + col);
                float4 kpn = zero4(), kp2r = zero4();
                if (KR) {
                    kp_q[ph % LA] = lds_(p.kap + (int64_t)(x + LA) * sx + col);
                    kp2r = ld4(p.kap + (int64_t)(x - M) * sx + col);   // for the second update
                } else {
                    kpn = lds_(p.kap + (int64_t)(x + 1) * sx + col);
                }
                ring[(ph + 2 * M + PF) % NQ] = ld4(p.cur + (int64_t)(x + M + PF) * sx + col);
                const float4 c = ring[(ph + M) % NQ];
                float* A = la + (x & 1) * LBA;
                float* U = lu + (x & 1) * LBU;
                float* arow = A + (ly + MY) * LWA;
                float* urow = U + ly * LWU;
                st4(arow + P + 4 * lz, ing ? c : zero4());
#pragma unroll
                for (int j = 0; j < JF; ++j)
                    if (hf_l[j] >= 0) st4(A + hf_l[j], hf_v[j] ? hf[j] : zero4());
                st4(urow + 4 * lz, uring[(ph + NQ - M) % NQ]);   // u^{n+1}(x - M)
                __syncthreads();

                // first update: u^{n+1}(x) on the extended tile
                {
                    float lap[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) lap[i] = p.c0 * comp(c, i);
#pragma unroll
                    for (int j = 1; j <= M; ++j) {
                        const float4 a = ring[(ph + M - j) % NQ], b = ring[(ph + M + j) % NQ];
                        lap[0] = fmaf(p.wx[j], a.x + b.x, lap[0]);
                        lap[1] = fmaf(p.wx[j], a.y + b.y, lap[1]);
                        lap[2] = fmaf(p.wx[j], a.z + b.z, lap[2]);
                        lap[3] = fmaf(p.wx[j], a.w + b.w, lap[3]);
                    }
#pragma unroll
                    for (int j = 1; j <= MY; ++j) {
                        const float4 a = ld4(arow - j * LWA + P + 4 * lz);
                        const float4 b = ld4(arow + j * LWA + P + 4 * lz);
                        lap[0] = fmaf(p.wy[j], a.x + b.x, lap[0]);
                        lap[1] = fmaf(p.wy[j], a.y + b.y, lap[1]);
                        lap[2] = fmaf(p.wy[j], a.z + b.z, lap[2]);
                        lap[3] = fmaf(p.wy[j], a.w + b.w, lap[3]);
                    }
                    {
                        float w[2 * P + 4];
#pragma unroll
                        for (int k = 0; k < (2 * P + 4) / 4; ++k) {
                            const float4 v = ld4(arow + 4 * lz + 4 * k);
                            w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int j = 1; j <= M; ++j)
                                lap[i] = fmaf(p.wz[j], w[P + i - j] + w[P + i + j], lap[i]);
                    }
                    const float ex = p.etax[min(max(x, 0), p.nx - 1)];
                    float4 o;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float v = update(comp(c, i), comp(uo, i), comp(kp, i), lap[i], ex + eyz[i], p.inv2dt);
                        if (z + i >= p.nz) v = 0.0f;
                        set_comp(o, i, v);
                    }
                    if (inj_nx[0] == x) {
                        const float4 inc = inj_nv[0];
                        o.x += inc.x; o.y += inc.y; o.z += inc.z; o.w += inc.w;
                        ++inj_i[0];
                        if (inj_i[0] < inj_e[0]) {
                            inj_nx[0] = inj_xl[0][inj_i[0]];
                            inj_nv[0] = inj_vl[0][inj_i[0]];
                        } else {
                            inj_nx[0] = INT_MAX;
                        }
                    }
                    if (!ing || x < 0 || x >= p.nx) o = zero4();
                    uring[ph % NQ] = o;
                }

                // second update: u^{n+2}(x - M) on the inner tile
                if (x >= xb + M && inner) {   // uniform in x; the z edge columns diverge
                    const int x2 = x - M;
                    const float4 c2 = uring[(ph + NQ - M) % NQ];
                    float lap[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) lap[i] = p.c0 * comp(c2, i);
#pragma unroll
                    for (int j = 1; j <= M; ++j) {
                        const float4 a = uring[(ph + NQ - M - j) % NQ], b = uring[(ph + NQ - M + j) % NQ];
                        lap[0] = fmaf(p.wx[j], a.x + b.x, lap[0]);
                        lap[1] = fmaf(p.wx[j], a.y + b.y, lap[1]);
                        lap[2] = fmaf(p.wx[j], a.z + b.z, lap[2]);
                        lap[3] = fmaf(p.wx[j], a.w + b.w, lap[3]);
                    }
#pragma unroll
                    for (int j = 1; j <= MY; ++j) {
                        const float4 a = ld4(urow - j * LWU + 4 * lz);
                        const float4 b = ld4(urow + j * LWU + 4 * lz);
                        lap[0] = fmaf(p.wy[j], a.x + b.x, lap[0]);
                        lap[1] = fmaf(p.wy[j], a.y + b.y, lap[1]);
                        lap[2] = fmaf(p.wy[j], a.z + b.z, lap[2]);
                        lap[3] = fmaf(p.wy[j], a.w + b.w, lap[3]);
                    }
                    {
                        float w[2 * P + 4];
#pragma unroll
                        for (int k = 0; k < (2 * P + 4) / 4; ++k) {
                            const float4 v = ld4(urow + 4 * lz - P + 4 * k);
                            w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int j = 1; j <= M; ++j)
                                lap[i] = fmaf(p.wz[j], w[P + i - j] + w[P + i + j], lap[i]);
                    }
                    const float4 uo2 = ring[ph % NQ];          // u^n(x - M)
                    const float4 kp2 = KR ? kp2r : kring[(ph + 1) % KQ];   // kap(x - M)
                    const float ex = p.etax[x2];
                    float4 o;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float v = update(comp(c2, i), comp(uo2, i), comp(kp2, i), lap[i], ex + eyz[i], p.inv2dt);
                        if (z + i >= p.nz) v = 0.0f;
                        set_comp(o, i, v);
                    }
                    if (inj_nx[1] == x2) {
                        const float4 inc = inj_nv[1];
                        o.x += inc.x; o.y += inc.y; o.z += inc.z; o.w += inc.w;
                        ++inj_i[1];
                        if (inj_i[1] < inj_e[1]) {
                            inj_nx[1] = inj_xl[1][inj_i[1]];
                            inj_nv[1] = inj_vl[1][inj_i[1]];
                        } else {
                            inj_nx[1] = INT_MAX;
                        }
                    }
                    if (ing) {
                        const int64_t base = (int64_t)x2 * sx;
                        st4o(p.out1 + base + col, c2);
                        st4o(p.out2 + base + col, o);
                    }
                }
                if (!KR) kring[(ph + 1) % KQ] = kpn;   // kap(x + 1), in the slot of kap(x - M)
            }
        }
    }
}

template <bool D3, int M, int BY, int BZE, int PF, int LA, bool KR, bool NTS>
__global__ void __launch_bounds__((BY + 2 * (D3 ? M : 0)) * BZE, D3 ? 1 : 3) k_step2(const Step2Params p) {
    step2_body<D3, M, BY, BZE, PF, LA, KR, NTS>(p, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// resident teams: one work-group steps one small grid held in LDS
// ---------------------------------------------------------------------------
// Dense LDS layout [x][y][zp], zp = z padded to 4 (the pad holds zeros).
// Every quantity is formed as in step_body, in the same order, so each node
// gets the same bits: lap = c0 c, then the x, y and z pairs (minus side
// first) by fmaf, then update(); the sources' increments (made by
// k_increments before the launch) are added after the update, the receivers
// interpolated from the field before it, in k_sample's corner order.
// Threads of a team: as many as keep every register of a thread's node
// column (the x ring, the z window, the plane ahead) without spilling:
// 1024 (16 waves, 128 VGPRs) for the 2D order-4 stencil, 256 for the 3D
// ones of order 12 and above, 512 otherwise.
__host__ __device__ constexpr int team_threads(bool d3, int m) {
    return d3 ? (m >= 6 ? 256 : 512) : (m <= 2 ? kTeamThreads : 512);
}

// How a shot is split over the work-groups of a team. Work-group w of W owns
// planes [w nx / W, (w + 1) nx / W) and holds K M more on either side (its
// window): for K updates it recomputes the part of its neighbours' planes
// that its own planes' stencils reach, on a window that narrows by M planes
// per update, and after every K updates the work-groups exchange K M
// boundary planes of the two newest fields through global memory with one
// barrier. The recomputed planes get the owners' bits (the same arithmetic
// on the same values), so the split changes no result. W = 1: one
// work-group holds the whole grid.
struct TeamPart {
    int w, W, K;
    float4* exch;               // [2 parities][W][2 sides][2 fields][K M planes][plane] (W > 1)
    unsigned int* cnt;          // the team's barrier counter (W > 1)
    unsigned int* err;          // raised when a barrier wait times out
    unsigned long long limit;   // longest barrier wait (s_memrealtime ticks, 100 MHz)
};

// Barrier of a team's work-groups: thread 0 arrives (release) and waits until
// `target` arrivals (then acquire). Every wait is bounded: on a timeout, or
// an error raised by another work-group, it raises the error and returns
// false, and the caller leaves.
__device__ bool team_sync(const TeamPart& tp, unsigned int target) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(tp.cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(tp.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(tp.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                __builtin_amdgcn_s_memrealtime() - t0 > tp.limit) {
                __hip_atomic_fetch_add(tp.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// A work item walks at least this many planes when there are enough: each
// item pays a set-up per update (column indices, ring fill, its first loads)
// that one plane does not amortise (measured on 141^2: 1.74 ms per 500
// updates split over 8 work-groups against 1.82 with one-plane items, 1.87
// with four).
constexpr int kTeamMinPlanes = 3;

template <bool D3, int M, bool SPLIT>
__device__ bool team_run(const TeamJob& J, float* F, const TeamPart& tp) {
    constexpr int T = team_threads(D3, M);
    constexpr int P = (M + 3) & ~3;
    constexpr int HZ = P / 4;
    constexpr int KS = D3 ? 8 : 4;   // corners of a receiver's cell
    const int tid = threadIdx.x;
    const int nx = J.nx, ny = J.ny, nz = J.nz;
    // the job's scalars, read once (uniform: scalar registers)
    const float c0 = J.c0, inv2dt = J.inv2dt;
    float wx[M + 1], wy[M + 1], wz[M + 1];
#pragma unroll
    for (int j = 1; j <= M; ++j) {
        wx[j] = J.wx[j];
        wy[j] = J.wy[j];
        wz[j] = J.wz[j];
    }
    const float* __restrict__ kap = J.kap;
    const float* __restrict__ etax = J.etax;
    const float* __restrict__ etay = J.etay;
    const float* __restrict__ etaz = J.etaz;
    const int64_t sxk = J.sx, syk = J.sy;
    const int nzv = (nz + 3) / 4;
    const int psx = ny * nzv;   // float4 per x plane
    // this work-group's planes [xs, xe) and the window [lo, hi) it holds
    const int W = SPLIT ? tp.W : 1;
    const int wr = SPLIT ? tp.w : 0;
    const int K = SPLIT ? tp.K : 1;
    const int KM = SPLIT ? K * M : 0;
    const int xs = wr * nx / W, xe = (wr + 1) * nx / W;
    const int lo = max(0, xs - KM), hi = min(nx, xe + KM);
    const int npts = (hi - lo) * psx * 4;
    float* A = F;          // u^n
    float* B = F + npts;   // u^{n-1}, overwritten by u^{n+1}
    for (int i = tid; i < 2 * npts; i += T) F[i] = 0.0f;
    const int ncol = psx;   // work items: a (y, z/4) column times a chunk of planes
    // pitched offset -> plane and dense index in the window, by float
    // reciprocals (a grid that fits has fewer than 2^24 pitched elements,
    // so the quotient estimate is off by at most one, which the remainder
    // test corrects)
    const int sxi = (int)J.sx, syi = (int)J.sy;
    const float rsx = 1.0f / (float)sxi, rsy = 1.0f / (float)syi;
    auto dense = [&](int64_t o64, int& xo) -> int {
        const int o = (int)o64;
        int x = (int)((float)o * rsx);
        int r = o - x * sxi;
        if (r < 0) {
            --x;
            r += sxi;
        } else if (r >= sxi) {
            ++x;
            r -= sxi;
        }
        int y = (int)((float)r * rsy);
        int z = r - y * syi;
        if (z < 0) {
            --y;
            z += syi;
        } else if (z >= syi) {
            ++y;
            z -= syi;
        }
        xo = x;
        return ((x - lo) * ny + y) * (nzv * 4) + z;
    };
    // the job's constant tables, converted once: the first receiver of each
    // thread (2D; 3D receivers are many and their registers are needed by
    // the stencil) and the first source node. A receiver belongs to the
    // work-group that owns its cell's first corner (the other corners lie in
    // its window); a source node is added by every work-group that computes
    // its plane, so that recomputed planes match their owner's.
    int rd[KS];
    float rw[KS];
    bool rown = false;
    if (!D3 && tid < J.nrec) {
        int xc = 0;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            int xk;
            rd[k] = dense(J.smp_off[(int64_t)tid * KS + k], xk);
            if (k == 0) xc = xk;
            rw[k] = J.smp_w[(int64_t)tid * KS + k];
        }
        rown = !SPLIT || (xc >= xs && xc < xe);
    }
    int nd = 0, ndx = 0;
    if (tid < J.nnodes) nd = dense(J.noff[tid], ndx);
    __syncthreads();
    auto sample = [&](const float* U, int row) {
        int i = tid;
        if (!D3 && i < J.nrec) {
            if (rown) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < KS; ++k) acc = fmaf(rw[k], U[rd[k]], acc);
                J.rec[(int64_t)row * J.nrec + i] = acc;
            }
            i += T;
        }
        for (; i < J.nrec; i += T) {
            int so[KS];
            float sw[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                so[k] = (int)J.smp_off[(int64_t)i * KS + k];
                sw[k] = J.smp_w[(int64_t)i * KS + k];
            }
            int xc = 0;
            int di[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                int xk;
                di[k] = dense(so[k], xk);
                if (k == 0) xc = xk;
            }
            if (SPLIT && (xc < xs || xc >= xe)) continue;
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < KS; ++k) acc = fmaf(sw[k], U[di[k]], acc);
            J.rec[(int64_t)row * J.nrec + i] = acc;
        }
    };
    for (int n = 0; n + 1 < J.nt; ++n) {
        // planes computed this update: the window narrowed by M per update
        // since the last exchange on every side that faces a neighbour
        const int j = SPLIT ? n % K : 0;
        const int clo = lo == 0 ? 0 : lo + (j + 1) * M;
        const int chi = hi == nx ? nx : hi - (j + 1) * M;
        const int ncomp = chi - clo;
        const int nch = max(1, min(T / ncol, ncomp / kTeamMinPlanes));
        // this update's increment of the thread's source node, used after
        // the update (its latency hides behind it)
        const bool inj = tid < J.nnodes && (!SPLIT || (ndx >= clo && ndx < chi));
        const float incv = inj ? J.inc[(int64_t)n * J.nnodes + tid] : 0.0f;
        sample(A, n);
        const float4* __restrict__ A4 = reinterpret_cast<const float4*>(A);
        float4* __restrict__ B4 = reinterpret_cast<float4*>(B);
        for (int item = tid; item < ncol * nch; item += T) {
            const int col = item % ncol, ch = item / ncol;
            const int y = col / nzv, zv = col - y * nzv, z = 4 * zv;
            const int x0 = clo + ch * ncomp / nch, x1 = clo + (ch + 1) * ncomp / nch;
            if (x0 >= x1) continue;
            const int cb = y * nzv + zv;   // the column in a plane (float4)
            // which z and y neighbour columns lie inside the grid (outside: zero)
            bool zok[2 * HZ + 1];
#pragma unroll
            for (int k = 0; k < 2 * HZ + 1; ++k) zok[k] = zv - HZ + k >= 0 && zv - HZ + k < nzv;
            bool ylo[M + 1], yhi[M + 1];
#pragma unroll
            for (int jj = 1; jj <= M; ++jj) {
                ylo[jj] = D3 && y - jj >= 0;
                yhi[jj] = D3 && y + jj < ny;
            }
            // x ring: planes x - M .. x + M of the column, and x + M + 1
            // loaded a plane ahead (planes outside the window are outside the
            // grid: zero); the walk is unrolled by the ring length, so every
            // slot index is a constant
            constexpr int NR = 2 * M + 2;
            float4 r[NR];
#pragma unroll
            for (int i = 0; i < 2 * M + 1; ++i) {
                const int xx = x0 - M + i;
                r[i] = xx >= lo && xx < hi ? A4[(xx - lo) * psx + cb] : zero4();
            }
            float eyz[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) eyz[i] = z + i < nz ? ((D3 ? etay[y] : 0.0f) + etaz[z + i]) : 0.0f;
            // kappa and eta_x of plane x + 1 are loaded while plane x is
            // computed (two slots; NR is even, so the slot is constant)
            const float* kcol = kap + (int64_t)y * syk + z;
            float4 kq[2];
            float eq[2];
            kq[0] = ld4(kcol + (int64_t)x0 * sxk);
            eq[0] = etax[x0];
            for (int xg = x0; xg < x1; xg += NR) {
#pragma unroll
                for (int ph = 0; ph < NR; ++ph) {
                    const int x = xg + ph;
                    if (x < x1) {
                        const int xn = x + M + 1;
                        r[(ph + 2 * M + 1) % NR] = xn < hi ? A4[(xn - lo) * psx + cb] : zero4();
                        if (x + 1 < x1) {
                            kq[(ph + 1) % 2] = ld4(kcol + (int64_t)(x + 1) * sxk);
                            eq[(ph + 1) % 2] = etax[x + 1];
                        }
                        const float4 kp = kq[ph % 2];
                        const float ex = eq[ph % 2];
                        const int pc = (x - lo) * psx + cb;
                        const float4 c = r[(ph + M) % NR];
                        float lap[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) lap[i] = c0 * comp(c, i);
#pragma unroll
                        for (int jj = 1; jj <= M; ++jj) {
                            const float4 a = r[(ph + M - jj) % NR], b = r[(ph + M + jj) % NR];
                            lap[0] = fmaf(wx[jj], a.x + b.x, lap[0]);
                            lap[1] = fmaf(wx[jj], a.y + b.y, lap[1]);
                            lap[2] = fmaf(wx[jj], a.z + b.z, lap[2]);
                            lap[3] = fmaf(wx[jj], a.w + b.w, lap[3]);
                        }
                        if (D3) {
#pragma unroll
                            for (int jj = 1; jj <= M; ++jj) {
                                const float4 a = ylo[jj] ? A4[pc - jj * nzv] : zero4();
                                const float4 b = yhi[jj] ? A4[pc + jj * nzv] : zero4();
                                lap[0] = fmaf(wy[jj], a.x + b.x, lap[0]);
                                lap[1] = fmaf(wy[jj], a.y + b.y, lap[1]);
                                lap[2] = fmaf(wy[jj], a.z + b.z, lap[2]);
                                lap[3] = fmaf(wy[jj], a.w + b.w, lap[3]);
                            }
                        }
                        {
                            float w[2 * P + 4];
#pragma unroll
                            for (int k = 0; k < 2 * HZ + 1; ++k) {
                                const float4 v = k == HZ ? c : (zok[k] ? A4[pc - HZ + k] : zero4());
                                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
                            }
#pragma unroll
                            for (int i = 0; i < 4; ++i)
#pragma unroll
                                for (int jj = 1; jj <= M; ++jj)
                                    lap[i] = fmaf(wz[jj], w[P + i - jj] + w[P + i + jj], lap[i]);
                        }
                        const float4 uo = B4[pc];
                        float4 o;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float v = update(comp(c, i), comp(uo, i), comp(kp, i), lap[i], ex + eyz[i], inv2dt);
                            if (z + i >= nz) v = 0.0f;
                            set_comp(o, i, v);
                        }
                        B4[pc] = o;
                    }
                }
            }
        }
        __syncthreads();
        // q^n into u^{n+1}: one thread per source node in the planes computed
        if (inj) B[nd] += incv;
        for (int k = tid + T; k < J.nnodes; k += T) {
            int xk;
            const int d = dense(J.noff[k], xk);
            if (!SPLIT || (xk >= clo && xk < chi)) B[d] += J.inc[(int64_t)n * J.nnodes + k];
        }
        if (SPLIT && (n + 1) % K == 0) {
            // u^{n+1} (B) and u^n (A) are now valid on the owned planes (and
            // u^n M planes beyond): exchange K M boundary planes of both with
            // the neighbours, double-buffered by exchange parity, so one
            // barrier per exchange separates a write from the reads of the
            // same buffer
            __syncthreads();
            const int e = (n + 1) / K;
            const int slab = KM * psx;
            float4* base = tp.exch + (int64_t)((e & 1) * W) * 4 * slab;
            float4* mine = base + (int64_t)wr * 4 * slab;   // [side][field][slab]
            float4* A4w = reinterpret_cast<float4*>(A);
            for (int i = tid; i < slab; i += T) {
                const int pl = i / psx, c = i - pl * psx;
                if (wr > 0) {
                    mine[i] = B4[(xs + pl - lo) * psx + c];
                    mine[slab + i] = A4w[(xs + pl - lo) * psx + c];
                }
                if (wr < W - 1) {
                    mine[2 * slab + i] = B4[(xe - KM + pl - lo) * psx + c];
                    mine[3 * slab + i] = A4w[(xe - KM + pl - lo) * psx + c];
                }
            }
            if (!team_sync(tp, (unsigned int)e * (unsigned int)W)) return false;
            const float4* left = base + (int64_t)(wr - 1) * 4 * slab + 2 * slab;   // its side 1
            const float4* right = base + (int64_t)(wr + 1) * 4 * slab;             // its side 0
            for (int i = tid; i < slab; i += T) {
                const int pl = i / psx, c = i - pl * psx;
                if (wr > 0) {
                    B4[(xs - KM + pl - lo) * psx + c] = left[i];
                    A4w[(xs - KM + pl - lo) * psx + c] = left[slab + i];
                }
                if (wr < W - 1) {
                    B4[(xe + pl - lo) * psx + c] = right[i];
                    A4w[(xe + pl - lo) * psx + c] = right[slab + i];
                }
            }
        }
        __syncthreads();
        float* t = A;
        A = B;
        B = t;
    }
    if (J.nt > 1) {
        sample(A, J.nt - 1);
    } else {
        for (int i = tid; i < J.nrec; i += T) {
            int xc;
            (void)dense(J.smp_off[(int64_t)i * KS], xc);
            if (!SPLIT || (xc >= xs && xc < xe)) J.rec[i] = 0.0f;
        }
    }
    return true;
}

__device__ inline bool team_fits_dev(int nx, int ny, int nz) {
    return nx > 0 && ny > 0 && nz > 0 && (int64_t)nx * ny * ((nz + 3) / 4 * 4) * 2 <= kTeamFieldFloats;
}

// A launch of resident teams. Width 1: work-groups take the launch's shots in
// order (one counter in device memory, zero at the launch), each stepping its
// shot to the end in LDS before it takes the next. Width W > 1: work-groups
// t W .. t W + W - 1 form team t, which steps shots t, t + teams, ... split
// over its W work-groups. The job is read from the table with a uniform
// index, so its scalars live in scalar registers.
template <bool D3, int M, bool SPLIT>
__global__ void __launch_bounds__(team_threads(D3, M), 1) k_team(const TeamArgs a) {
    __shared__ __attribute__((aligned(16))) float F[kTeamFieldFloats];
    __shared__ int s_j;
    const TeamJob* __restrict__ jobs = a.jobs;
    const int W = SPLIT ? a.width : 1;
    auto valid = [&](const TeamJob& J) {
        // the host groups shots by (ndim, half), admits only grids that fit
        // and splits a grid only where every part keeps at least K M planes;
        // a table entry that does not hold is skipped rather than overrun LDS
        return J.ndim == (D3 ? 3 : 2) && J.half == M && team_fits_dev(J.nx, J.ny, J.nz) &&
               (!SPLIT || (a.period >= 1 && J.nx / W >= a.period * M));
    };
    if (!SPLIT) {
        const TeamPart tp{0, 1, 1, nullptr, nullptr, a.err, a.limit};
        for (;;) {
            if (threadIdx.x == 0) s_j = (int)atomicAdd(a.next, 1u);
            __syncthreads();
            const int j = __builtin_amdgcn_readfirstlane(s_j);
            __syncthreads();   // s_j is rewritten for the next shot
            if (j >= a.njobs) return;   // uniform
            const TeamJob& J = jobs[j];
            if (valid(J)) (void)team_run<D3, M, false>(J, F, tp);
            __syncthreads();   // F is cleared for the next shot
        }
    } else {
        const int team = blockIdx.x / W, nteams = gridDim.x / W;
        if (team >= nteams) return;
        for (int j = team; j < a.njobs; j += nteams) {
            const TeamJob& J = jobs[j];
            const TeamPart tp{(int)(blockIdx.x % W), W, a.period, a.exch + (int64_t)j * a.exch_stride,
                              a.cnt + (int64_t)j * 32, a.err, a.limit};
            if (valid(J) && !team_run<D3, M, true>(J, F, tp)) return;   // a barrier timed out
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// sparse operators and helpers
// ---------------------------------------------------------------------------
__global__ void k_inject(const InjectParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.nnodes) return;
    float acc = 0.0f;
    for (int e = p.seg[i]; e < p.seg[i + 1]; ++e) acc = fmaf(p.w[e], p.vals[p.pt[e]], acc);
    const int64_t o = p.off[i];
    const float k = p.kap[o];
    const float g = p.eta[i] * k * p.inv2dt;
    const float inc = acc * (k * __builtin_amdgcn_rcpf(1.0f + g));
    p.field[o] += inc;
    if (p.grad) p.grad[o] -= p.ufwd[o] * inc * p.idt2;
}

__global__ void k_increments(const IncParams p) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (k >= p.nnodes) return;
    const float kk = p.kap[p.off[k]];
    const float g = p.eta[k] * kk * p.inv2dt;
    const float scale = kk * __builtin_amdgcn_rcpf(1.0f + g);
    for (int row = n; row < p.nrows; row += gridDim.y) {
        const float* v = p.vals + (int64_t)row * p.npts;
        float acc = 0.0f;
        for (int e = p.seg[k]; e < p.seg[k + 1]; ++e) acc = fmaf(p.w[e], v[p.pt[e]], acc);
        p.inc[(int64_t)row * p.nnodes + k] = acc * scale;
    }
}

__global__ void k_sample(const float* __restrict__ field, const int64_t* __restrict__ off,
                         const float* __restrict__ w, int npts, int K, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) acc = fmaf(w[i * K + k], field[off[i * K + k]], acc);
    out[i] = acc;
}

// Row-wise kernels over the nx*ny rows of a field: blockIdx.y strides over rows
// (the y grid dimension is limited to 65535), threads over z.
__global__ void k_coef(const float* __restrict__ m, float* __restrict__ kap, int nx, int ny,
                       int nz, int64_t sx, int64_t sy, double dt2) {
    const int64_t nrows = (int64_t)nx * ny;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y) {
        const int x = (int)(row / ny), y = (int)(row % ny);
        for (int z = blockIdx.x * blockDim.x + threadIdx.x; z < sy; z += gridDim.x * blockDim.x) {
            float v = 0.0f;
            if (z < nz) v = (float)(dt2 / (double)m[row * nz + z]);
            kap[(int64_t)x * sx + (int64_t)y * sy + z] = v;
        }
    }
}

__global__ void k_unpitch(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny,
                          int nz, int64_t sx, int64_t sy) {
    const int64_t nrows = (int64_t)nx * ny;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y) {
        const int x = (int)(row / ny), y = (int)(row % ny);
        for (int z = blockIdx.x * blockDim.x + threadIdx.x; z < nz; z += gridDim.x * blockDim.x)
            dst[row * nz + z] = src[(int64_t)x * sx + (int64_t)y * sy + z];
    }
}

__global__ void k_pitch(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny,
                        int nz, int64_t sx, int64_t sy) {
    const int64_t nrows = (int64_t)nx * ny;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y) {
        const int x = (int)(row / ny), y = (int)(row % ny);
        for (int z = blockIdx.x * blockDim.x + threadIdx.x; z < sy; z += gridDim.x * blockDim.x)
            dst[(int64_t)x * sx + (int64_t)y * sy + z] = z < nz ? src[row * nz + z] : 0.0f;
    }
}

__global__ void k_fill(float* __restrict__ d, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = v;
}


__global__ void k_residual(const float* d, const float* __restrict__ d_obs, float* r, int64_t n,
                           double* partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = d[i] - d_obs[i];
        r[i] = v;
        acc += (double)v * (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_count_nonfinite(const float* __restrict__ x, int64_t n, unsigned int* count) {
    unsigned int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += isfinite(x[i]) ? 0u : 1u;
    if (c) atomicAdd(count, c);
}

// out2[0] = bits of the smallest positive value, out2[1] = bits of the largest,
// out2[2] = number of values that are not positive and finite. For positive
// finite floats the IEEE bit pattern orders like the value.
__global__ void k_minmax(const float* __restrict__ x, int64_t n, unsigned int* out3) {
    unsigned int lo = 0x7f7fffffu, hi = 0u, bad = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[i];
        if (!(v > 0.0f) || !isfinite(v)) { ++bad; continue; }
        const unsigned int b = __float_as_uint(v);
        lo = min(lo, b);
        hi = max(hi, b);
    }
    atomicMin(&out3[0], lo);
    atomicMax(&out3[1], hi);
    if (bad) atomicAdd(&out3[2], bad);
}

__global__ void k_strip(float* __restrict__ field, float* __restrict__ strip, const StripGeom g,
                        int to_field) {
    const int64_t n = g.start[g.nslab];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < g.nslab && i >= g.start[k + 1]) ++k;
        const int64_t j = i - g.start[k];
        const int64_t ez = g.z1[k] - g.z0[k], ey = g.y1[k] - g.y0[k];
        const int64_t z = g.z0[k] + j % ez;
        const int64_t t = j / ez;
        const int64_t y = g.y0[k] + t % ey;
        const int64_t x = g.x0[k] + t / ey;
        const int64_t o = x * g.sx + y * g.sy + z;
        if (to_field) field[o] = strip[i];
        else strip[i] = field[o];
    }
}

__global__ void k_mask_box(float* __restrict__ f, int nx, int ny, int nz, int64_t sx, int64_t sy,
                           int bx0, int bx1, int by0, int by1, int bz0, int bz1) {
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % nz);
        const int64_t t = i / nz;
        const int y = (int)(t % ny);
        const int x = (int)(t / ny);
        if (x < bx0 || x >= bx1 || y < by0 || y >= by1 || z < bz0 || z >= bz1)
            f[(int64_t)x * sx + (int64_t)y * sy + z] = 0.0f;
    }
}

__global__ void k_update(float* __restrict__ m, const float* __restrict__ g, float alpha, float lo,
                         float hi, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m[i] = fminf(fmaxf(fmaf(-alpha, g[i], m[i]), lo), hi);
}

unsigned rows_grid(int nx, int ny) {
    return (unsigned)std::min<int64_t>((int64_t)nx * ny, 65535);
}

int grid_1d(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

#ifndef WF_PF_LO
#define WF_PF_LO 1
#endif
#ifndef WF_PF_HI
#define WF_PF_HI 1
#endif

// Compiled 3D tile shapes (z threads x y threads): 128 x 8 nodes, whose rows
// are whole 128-byte lines on line-aligned rows, and 64 x 16 nodes for thin
// grids (fewer than 96 nodes along z). Measured on the 336^3 order-8 step,
// 128 x 8 moves ~12% less data than 64 x 16 and ~8% less than 112 x 8.
constexpr TileShape kTiles3[2] = {{32, 8}, {16, 16}};
// 2D: one row of 256 z nodes per block, or 512 for long rows (measured on
// 8272^2 order 8: 208 us per update against 245 us with 256).
constexpr TileShape kTiles2[2] = {{64, 1}, {128, 1}};

template <int M, int T, int MODE>
const void* step3_fn() {
    constexpr int PF = M <= 4 ? WF_PF_LO : WF_PF_HI;
    return reinterpret_cast<const void*>(&k_step<true, M, kTiles3[T].bz, kTiles3[T].by, PF, MODE>);
}
template <int M, int T, int MODE>
const void* step2_fn() {
    constexpr int PF = M <= 4 ? WF_PF_LO : WF_PF_HI;
    return reinterpret_cast<const void*>(&k_step<false, M, kTiles2[T].bz, kTiles2[T].by, PF, MODE>);
}

template <int M, int MODE>
const void* step_fn_mm(int ndim, int tile) {
    if (ndim == 2) return tile == 1 ? step2_fn<M, 1, MODE>() : step2_fn<M, 0, MODE>();
    if (tile == 0) return step3_fn<M, 0, MODE>();
    return step3_fn<M, 1, MODE>();
}

template <int M>
const void* step_fn_m(int ndim, int tile, int mode) {
    switch (mode) {
        case kModePlain: return step_fn_mm<M, kModePlain>(ndim, tile);
        case kModeImaging: return step_fn_mm<M, kModeImaging>(ndim, tile);
        case kModeBornSource: return step_fn_mm<M, kModeBornSource>(ndim, tile);
        case kModeVolumeSource: return step_fn_mm<M, kModeVolumeSource>(ndim, tile);
        default: return nullptr;
    }
}

const void* step_fn(int ndim, int half, int tile, int mode) {
    switch (half) {
        case 2: return step_fn_m<2>(ndim, tile, mode);
        case 3: return step_fn_m<3>(ndim, tile, mode);
        case 4: return step_fn_m<4>(ndim, tile, mode);
        case 5: return step_fn_m<5>(ndim, tile, mode);
        case 6: return step_fn_m<6>(ndim, tile, mode);
        case 7: return step_fn_m<7>(ndim, tile, mode);
        case 8: return step_fn_m<8>(ndim, tile, mode);
        default: return nullptr;
    }
}

int step_capacity(int ndim, int half, int tile, int mode) {
    static std::mutex mu;
    static int cache[2][kMaxHalf + 1][2][kModeCount] = {};
    static int cus = 0;
    std::lock_guard<std::mutex> lk(mu);
    int& c = cache[ndim - 2][half][tile][mode];
    if (c > 0) return c;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    const TileShape ts = step_tile(ndim, tile);
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step_fn(ndim, half, tile, mode),
                                                     ts.bz * ts.by, 0) != hipSuccess ||
        per < 1)
        per = 1;
    // The chunk plan assumes at most 12 resident waves per CU (3 blocks of 4
    // waves): planning for 16 gave more, shorter chunks, whose extra warm-up
    // planes cost 10% on the 336^3 order-8 step. (The hardware may still place
    // a fourth block; capping residency with unused LDS changed nothing.)
    const int waves = ts.bz * ts.by / 64;
    int max_waves = 12;
    if (const char* e = std::getenv("WAVEFD_WAVES_PER_CU")) max_waves = std::max(1, std::atoi(e));
    per = std::min(per, std::max(1, max_waves / std::max(1, waves)));
    c = per * cus;
    return c;
}

}  // namespace

TileShape step_tile(int ndim, int tile) {
    if (ndim == 3) return kTiles3[tile == 1 ? 1 : 0];
    return kTiles2[tile == 1 ? 1 : 0];
}

void step_plan(StepParams& p, int ndim, int half, int mode, int cx_request, int tile_request) {
    int tile = 0;
    if (tile_request == 0 || tile_request == 1) {
        tile = tile_request;
    } else if (ndim == 3) {
        tile = p.nz < 96 ? 1 : 0;
    } else {
        tile = p.nz >= 1024 ? 1 : 0;
    }
    p.tile = tile;
    const TileShape ts = step_tile(ndim, tile);
    const int tz = 4 * ts.bz;
    p.ntz = (p.nz + tz - 1) / tz;
    p.nty = ndim == 3 ? (p.ny + ts.by - 1) / ts.by : 1;
    const int64_t tiles = (int64_t)p.ntz * p.nty;
    int cx = cx_request;
    if (cx <= 0) {
        // Chunks along x trade parallelism against the 2M + PF planes every
        // chunk re-reads to fill its register ring. Cost model per resident
        // round of blocks: (planes + warm-up) / occupancy, times the rounds,
        // plus kRoundPlanes planes per round beyond the first: blocks of a
        // later round start out of step with their neighbours (whose rows
        // they read as halos) and with the other x positions in flight (the
        // same walk with no stencil at 592^3 took 615 us in one round of 740
        // blocks and 645 us in two rounds of 1480; the step kernel 663 and
        // 680 us at order 8).
        constexpr double kRoundPlanes = 8.0;
        const int cap = step_capacity(ndim, half, tile, mode);
        const int warm = 2 * half + 1;
        double best = 1e300;
        int best_n = 1;
        for (int n = 1; n <= p.nx; ++n) {
            const int c = (p.nx + n - 1) / n;
            if (n > 1 && (p.nx + c - 1) / c != n) continue;   // same chunking as a smaller n
            const double blocks = (double)tiles * n;
            const double rounds = std::ceil(blocks / cap);
            const double fill = std::min(1.0, blocks / cap);
            const double cost = rounds * (c + warm) / fill + (rounds - 1) * kRoundPlanes;
            if (cost < best * 0.999) {
                best = cost;
                best_n = n;
            }
        }
        cx = (p.nx + best_n - 1) / best_n;
    }
    p.cx = std::min(cx, p.nx);
    p.nchunks = (p.nx + p.cx - 1) / p.cx;
    p.nblocks = (int)(tiles * p.nchunks);
}

hipError_t launch_step(const StepParams& p, int ndim, int half, int mode, hipStream_t s) {
    if (p.nblocks <= 0) return hipSuccess;
    const void* fn = step_fn(ndim, half, p.tile, mode);
    if (!fn) return hipErrorInvalidValue;
    const TileShape ts = step_tile(ndim, p.tile);
    const int grid = ((p.nblocks + 7) / 8) * 8;
    void* args[] = {const_cast<StepParams*>(&p)};
    return hipLaunchKernel(fn, dim3(grid), dim3(ts.bz * ts.by), args, 0, s);
}

// Two-update kernel: 24 extended rows of 32 float4 columns (768 threads),
// i.e. 20 inner rows at order 4 and 16 at order 8, one block per CU (its two
// rings and the LDS reads in flight hold about 165 VGPRs); the u^n ring
// prefetches one plane. Per order, as measured at 592^3 (us per launch of
// two updates): order 4 with u^{n-1} and kap cached (neighbouring blocks
// re-read the rows their extended tiles share: 1129 against 1195 streamed,
// 16 inner rows) and 20 inner rows (1076; 16 rows recompute a larger share);
// order 8 also reloading kap for the second update instead of keeping a ring
// of it (1424 against 1525: the ring spilled), 16 inner rows (12: 1473); a
// deeper prefetch spilled more and was slower.
constexpr int step2_rows(int half) { return half == 2 ? 20 : 16; }
// Measured against two single-update launches (us per update, constant
// velocity, 40 updates): order 4 gains 1.13-1.21 x from 464^3 (1.0e8 nodes)
// to 592^3; below that the result swings with how the 120-node z tiles and
// 20-row y tiles fill the grid and how many rounds of blocks the chunking
// needs (400^3 1.07 x, 432^3 0.99 x, 368^3 0.73 x with a last z tile of 8
// nodes, 272^3 to 336^3 0.89-0.96 x where the single-update kernel also
// finds much of its traffic in the Infinity Cache); order 8 is bound by
// instruction issue (every tile recomputes u^{n+1} on a margin of M rows and
// 4 nodes) and loses at every size from 208^3 to 592^3 (0.76-0.93 x).
constexpr int64_t kStep2MinNodes = 90000000;

// 2D rows: 128 float4 columns (504 inner nodes along z), two waves per
// block and several blocks per CU; the margin is 4 z nodes per side, so
// the recomputed work is under 2 %. Measured against one update per launch
// (constant velocity, nbl 20-40): order 4 gains at every size from 141^2
// (3.35 against 3.99 us per update: half the launches) to 8272^2 (1.04-1.38
// x); order 8 loses from 141^2 to 1448^2 (0.78-0.86 x: the stencil's
// issue time per launch exceeds the launch it saves), breaks even at 2896^2
// and 5792^2 (1.02, 0.97 x) and gains 1.30 x at 8272^2 (6.8e7 nodes), where
// a single-update launch no longer finds its fields in the Infinity Cache.
constexpr int64_t kStep2MinNodes2dOrder8 = 50000000;

namespace {
const void* step2_fn(int ndim, int half) {
    constexpr int C3 = step2_cols(true), C2 = step2_cols(false);
    if (ndim == 3) {
        switch (half) {
            case 2: return reinterpret_cast<const void*>(&k_step2<true, 2, step2_rows(2), C3, 1, 1, false, false>);
            case 4: return reinterpret_cast<const void*>(&k_step2<true, 4, step2_rows(4), C3, 1, 1, true, false>);
            default: return nullptr;
        }
    }
    if (ndim == 2) {
        switch (half) {
            case 2: return reinterpret_cast<const void*>(&k_step2<false, 2, 1, C2, 1, 1, false, false>);
            case 4: return reinterpret_cast<const void*>(&k_step2<false, 4, 1, C2, 1, 1, true, false>);
            default: return nullptr;
        }
    }
    return nullptr;
}
int step2_by(int ndim, int half) { return ndim == 3 ? step2_rows(half) : 1; }
}  // namespace

bool step2_supported(int ndim, int half) { return step2_fn(ndim, half) != nullptr; }
bool step2_preferred(int ndim, int half, int64_t nodes) {
    if (!step2_supported(ndim, half)) return false;
    if (ndim == 2) return half == 2 || nodes >= kStep2MinNodes2dOrder8;
    return half == 2 && nodes >= kStep2MinNodes;
}
int step2_ext_cols(int half) { return (half + 3) / 4; }
int step2_threads(int ndim, int half, int by) {
    return (by + (ndim == 3 ? 2 * half : 0)) * step2_cols(ndim == 3);
}

void step2_plan(Step2Params& p, int ndim, int half, int cx_request) {
    static std::mutex mu;
    static int cap_cache[2][kMaxHalf + 1] = {};
    p.by = step2_by(ndim, half);
    const int tz = 4 * (step2_cols(ndim == 3) - 2 * step2_ext_cols(half));
    p.ntz = (p.nz + tz - 1) / tz;
    p.nty = (p.ny + p.by - 1) / p.by;
    const int64_t tiles = (int64_t)p.ntz * p.nty;
    int cap = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        int& cc = cap_cache[ndim == 3][half];
        if (cc <= 0) {
            int dev = 0, cus = 0, per = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                cus = 256;
            const void* fn = step2_fn(ndim, half);
            if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, step2_threads(ndim, half, p.by), 0) !=
                           hipSuccess || per < 1)
                per = 1;
            cc = per * cus;
        }
        cap = cc;
    }
    int cx = cx_request;
    if (cx <= 0) {
        // as step_plan: every chunk walks 2M planes beyond its own (the
        // first update's extension), rounds beyond the first cost kRoundPlanes
        constexpr double kRoundPlanes = 8.0;
        const int warm = 2 * half;
        double best = 1e300;
        int best_n = 1;
        for (int n = 1; n <= p.nx; ++n) {
            const int c = (p.nx + n - 1) / n;
            if (n > 1 && (p.nx + c - 1) / c != n) continue;
            const double blocks = (double)tiles * n;
            const double rounds = std::ceil(blocks / cap);
            const double fill = std::min(1.0, blocks / cap);
            const double cost = rounds * (c + warm) / fill + (rounds - 1) * kRoundPlanes;
            if (cost < best * 0.999) {
                best = cost;
                best_n = n;
            }
        }
        cx = (p.nx + best_n - 1) / best_n;
    }
    p.cx = std::max(1, std::min(cx, p.nx));
    p.nchunks = (p.nx + p.cx - 1) / p.cx;
    p.nblocks = (int)(tiles * p.nchunks);
}

hipError_t launch_step2(const Step2Params& p, int ndim, int half, hipStream_t s) {
    if (p.nblocks <= 0) return hipSuccess;
    const void* fn = step2_fn(ndim, half);
    if (!fn || p.by != step2_by(ndim, half)) return hipErrorInvalidValue;
    const int grid = ((p.nblocks + 7) / 8) * 8;
    void* args[] = {const_cast<Step2Params*>(&p)};
    return hipLaunchKernel(fn, dim3(grid), dim3(step2_threads(ndim, half, p.by)), args, 0, s);
}

template <int M>
hipError_t launch_batch_m(const BatchJob* jobs, int njobs, int total, int ndim, int tile, int k,
                          hipStream_t s) {
    constexpr int PF = M <= 4 ? WF_PF_LO : WF_PF_HI;
    if (ndim == 2 && tile == 1) {
        hipLaunchKernelGGL((k_step_batch<false, M, kTiles2[1].bz, kTiles2[1].by, PF>), dim3(total),
                           dim3(kTiles2[1].bz * kTiles2[1].by), 0, s, jobs, njobs, k);
    } else if (ndim == 2) {
        hipLaunchKernelGGL((k_step_batch<false, M, kTiles2[0].bz, kTiles2[0].by, PF>), dim3(total),
                           dim3(kTiles2[0].bz * kTiles2[0].by), 0, s, jobs, njobs, k);
    } else if (tile == 0) {
        hipLaunchKernelGGL((k_step_batch<true, M, kTiles3[0].bz, kTiles3[0].by, PF>), dim3(total),
                           dim3(kTiles3[0].bz * kTiles3[0].by), 0, s, jobs, njobs, k);
    } else {
        hipLaunchKernelGGL((k_step_batch<true, M, kTiles3[1].bz, kTiles3[1].by, PF>), dim3(total),
                           dim3(kTiles3[1].bz * kTiles3[1].by), 0, s, jobs, njobs, k);
    }
    return hipGetLastError();
}

hipError_t launch_step_batch(const BatchJob* jobs, int njobs, int total, int ndim, int half, int tile,
                             int k, hipStream_t s) {
    if (njobs <= 0 || total <= 0) return hipSuccess;
    switch (half) {
        case 2: return launch_batch_m<2>(jobs, njobs, total, ndim, tile, k, s);
        case 3: return launch_batch_m<3>(jobs, njobs, total, ndim, tile, k, s);
        case 4: return launch_batch_m<4>(jobs, njobs, total, ndim, tile, k, s);
        case 5: return launch_batch_m<5>(jobs, njobs, total, ndim, tile, k, s);
        case 6: return launch_batch_m<6>(jobs, njobs, total, ndim, tile, k, s);
        case 7: return launch_batch_m<7>(jobs, njobs, total, ndim, tile, k, s);
        case 8: return launch_batch_m<8>(jobs, njobs, total, ndim, tile, k, s);
        default: return hipErrorInvalidValue;
    }
}

bool team_fits(int64_t nx, int64_t ny, int64_t nz) {
    return nx > 0 && ny > 0 && nz > 0 && nx * ny * ((nz + 3) / 4 * 4) * 2 <= kTeamFieldFloats;
}

template <bool D3, bool SPLIT>
hipError_t launch_team_d(const TeamArgs& a, int half, int nwg, hipStream_t s) {
    const dim3 g(nwg);
    switch (half) {
        case 2: hipLaunchKernelGGL((k_team<D3, 2, SPLIT>), g, dim3(team_threads(D3, 2)), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_team<D3, 3, SPLIT>), g, dim3(team_threads(D3, 3)), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_team<D3, 4, SPLIT>), g, dim3(team_threads(D3, 4)), 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_team<D3, 5, SPLIT>), g, dim3(team_threads(D3, 5)), 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_team<D3, 6, SPLIT>), g, dim3(team_threads(D3, 6)), 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_team<D3, 7, SPLIT>), g, dim3(team_threads(D3, 7)), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_team<D3, 8, SPLIT>), g, dim3(team_threads(D3, 8)), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_team(const TeamArgs& a, int ndim, int half, int nwg, hipStream_t s) {
    if (nwg <= 0) return hipSuccess;
    if (a.width > 1) {
        if (nwg % a.width != 0 || a.period < 1) return hipErrorInvalidValue;
        return ndim == 3 ? launch_team_d<true, true>(a, half, nwg, s) : launch_team_d<false, true>(a, half, nwg, s);
    }
    return ndim == 3 ? launch_team_d<true, false>(a, half, nwg, s) : launch_team_d<false, false>(a, half, nwg, s);
}

hipError_t launch_inject(const InjectParams& p, hipStream_t s) {
    if (p.nnodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject, dim3((p.nnodes + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_increments(const IncParams& p, hipStream_t s) {
    if (p.nnodes <= 0 || p.nrows <= 0) return hipSuccess;
    dim3 g((p.nnodes + 255) / 256, (unsigned)std::min(p.nrows, 4096));
    hipLaunchKernelGGL(k_increments, g, dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_sample(const float* field, const int64_t* off, const float* w, int npts, int K,
                         float* out, hipStream_t s) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample, dim3((npts + 255) / 256), dim3(256), 0, s, field, off, w, npts, K,
                       out);
    return hipGetLastError();
}

hipError_t launch_coef(const float* m, float* kap, int nx, int ny, int nz, int64_t sx, int64_t sy,
                       double dt, hipStream_t s) {
    dim3 g((unsigned)std::min<int64_t>((sy + 255) / 256, 64), rows_grid(nx, ny));
    hipLaunchKernelGGL(k_coef, g, dim3(256), 0, s, m, kap, nx, ny, nz, sx, sy, dt * dt);
    return hipGetLastError();
}

hipError_t launch_unpitch(const float* src, float* dst, int nx, int ny, int nz, int64_t sx,
                          int64_t sy, hipStream_t s) {
    dim3 g((unsigned)std::min<int64_t>((nz + 255) / 256, 64), rows_grid(nx, ny));
    hipLaunchKernelGGL(k_unpitch, g, dim3(256), 0, s, src, dst, nx, ny, nz, sx, sy);
    return hipGetLastError();
}

hipError_t launch_pitch(const float* src, float* dst, int nx, int ny, int nz, int64_t sx,
                        int64_t sy, hipStream_t s) {
    dim3 g((unsigned)std::min<int64_t>((sy + 255) / 256, 64), rows_grid(nx, ny));
    hipLaunchKernelGGL(k_pitch, g, dim3(256), 0, s, src, dst, nx, ny, nz, sx, sy);
    return hipGetLastError();
}

hipError_t launch_fill(float* dst, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n, 256)), dim3(256), 0, s, dst, n, v);
    return hipGetLastError();
}

int residual_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024)); }

hipError_t launch_residual(const float* d, const float* d_obs, float* r, int64_t n, double* partial,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(residual_blocks(n)), dim3(256), 0, s, d, d_obs, r, n, partial);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* x, int64_t n, unsigned int* count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_1d(n, 256)), dim3(256), 0, s, x, n, count);
    return hipGetLastError();
}

hipError_t launch_strip(float* field, float* strip, const StripGeom& g, int to_field, hipStream_t s) {
    const int64_t n = g.start[g.nslab];
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_strip, dim3(grid_1d(n, 256)), dim3(256), 0, s, field, strip, g, to_field);
    return hipGetLastError();
}

hipError_t launch_mask_box(float* field, int nx, int ny, int nz, int64_t sx, int64_t sy, int bx0,
                           int bx1, int by0, int by1, int bz0, int bz1, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_box, dim3(grid_1d(n, 256)), dim3(256), 0, s, field, nx, ny, nz, sx, sy,
                       bx0, bx1, by0, by1, bz0, bz1);
    return hipGetLastError();
}

hipError_t launch_update(float* m, const float* g, float alpha, float lo, float hi, int64_t n,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update, dim3(grid_1d(n, 256)), dim3(256), 0, s, m, g, alpha, lo, hi, n);
    return hipGetLastError();
}

hipError_t launch_minmax(const float* x, int64_t n, float* out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minmax, dim3(grid_1d(n, 256)), dim3(256), 0, s, x, n,
                       reinterpret_cast<unsigned int*>(out3));
    return hipGetLastError();
}

}  // namespace wf
