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

namespace wf {

namespace {

__device__ __forceinline__ float4 ld4(const float* p) {
    return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ void st4(float* p, const float4& v) {
    *reinterpret_cast<float4*>(p) = v;
}
__device__ __forceinline__ float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }
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

// One point's update, given its Laplacian.
__device__ __forceinline__ float update(float c, float old, float kap, float lap, float eta,
                                        float inv2dt) {
    const float g = eta * kap * inv2dt;
    const float num = fmaf(kap, lap, fmaf(g, old, 2.0f * c - old));
    return num * __builtin_amdgcn_rcpf(1.0f + g);
}

// ---------------------------------------------------------------------------
// 3D step. Block: BZ x BY threads, tile TZ = 4 BZ (z) by BY (y).
// ---------------------------------------------------------------------------
template <int M, int BZ, int BY, bool IMG>
__global__ void __launch_bounds__(BZ * BY) k_step3d(const StepParams p) {
    constexpr int NT = BZ * BY;
    constexpr int TZ = 4 * BZ;
    constexpr int P = (M + 3) & ~3;     // z halo rounded up to whole float4s
    constexpr int HZ = P / 4;
    constexpr int LW = TZ + 2 * P;      // LDS row (floats)
    constexpr int LH = BY + 2 * M;      // LDS rows
    __shared__ __attribute__((aligned(16))) float lds[LH * LW];

    const int r = xcd_remap(blockIdx.x, p.nblocks);
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
    const int64_t col = own ? (int64_t)y * p.sy + z : 0;

    float eyz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        eyz[i] = (own && z + i < p.nz) ? (p.etay[y] + p.etaz[z + i]) : 0.0f;

    float4 q[2 * M + 1];
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) {
        const int xx = xb - M + j;
        q[j] = (own && xx >= 0 && xx < p.nx) ? ld4(p.cur + (int64_t)xx * p.sx + col) : zero4();
    }
    float* lrow = lds + (ly + M) * LW;

    for (int x = xb; x < xe; ++x) {
        const int64_t base = (int64_t)x * p.sx;
        {
            const int xn = x + M;
            q[2 * M] = (own && xn < p.nx) ? ld4(p.cur + (int64_t)xn * p.sx + col) : zero4();
        }
        const float4 uo = own ? ld4(p.old + base + col) : zero4();
        const float4 kp = own ? ld4(p.kap + base + col) : zero4();
        float4 uf = zero4(), gr = zero4();
        if (IMG && own) {
            uf = ld4(p.ufwd + base + col);
            gr = ld4(p.grad + base + col);
        }
        const float ex = p.etax[x];

        // stage the plane: own centre, y halo rows, z halo columns
        st4(lrow + P + 4 * lz, q[M]);
        for (int i = tid; i < 2 * M * BZ; i += NT) {
            const int rr = i / BZ, cz = i - rr * BZ;
            const int lr = rr < M ? rr : rr + BY;
            const int gy = y0 - M + lr;
            const int gz = z0 + 4 * cz;
            float4 v = zero4();
            if (gy >= 0 && gy < p.ny && gz < p.nz) v = ld4(p.cur + base + (int64_t)gy * p.sy + gz);
            st4(lds + lr * LW + P + 4 * cz, v);
        }
        for (int i = tid; i < 2 * BY * HZ; i += NT) {
            const int rr = i / (2 * HZ), k = i - rr * (2 * HZ);
            const int side = k / HZ, kk = k - side * HZ;
            const int lc = side ? (P + TZ + 4 * kk) : 4 * kk;
            const int gz = z0 - P + lc;
            const int gy = y0 + rr;
            float4 v = zero4();
            if (gy < p.ny && gz >= 0 && gz < p.nz) v = ld4(p.cur + base + (int64_t)gy * p.sy + gz);
            st4(lds + (rr + M) * LW + lc, v);
        }
        __syncthreads();

        float lap[4];
        {
            const float4 c = q[M];
#pragma unroll
            for (int i = 0; i < 4; ++i) lap[i] = p.c0 * comp(c, i);
#pragma unroll
            for (int j = 1; j <= M; ++j) {
                const float4 a = q[M - j], b = q[M + j];
                lap[0] = fmaf(p.wx[j], a.x + b.x, lap[0]);
                lap[1] = fmaf(p.wx[j], a.y + b.y, lap[1]);
                lap[2] = fmaf(p.wx[j], a.z + b.z, lap[2]);
                lap[3] = fmaf(p.wx[j], a.w + b.w, lap[3]);
            }
#pragma unroll
            for (int j = 1; j <= M; ++j) {
                const float4 a = ld4(lds + (ly + M - j) * LW + P + 4 * lz);
                const float4 b = ld4(lds + (ly + M + j) * LW + P + 4 * lz);
                lap[0] = fmaf(p.wy[j], a.x + b.x, lap[0]);
                lap[1] = fmaf(p.wy[j], a.y + b.y, lap[1]);
                lap[2] = fmaf(p.wy[j], a.z + b.z, lap[2]);
                lap[3] = fmaf(p.wy[j], a.w + b.w, lap[3]);
            }
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

        float4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = update(comp(q[M], i), comp(uo, i), comp(kp, i), lap[i], ex + eyz[i], p.inv2dt);
            if (z + i >= p.nz) v = 0.0f;
            set_comp(o, i, v);
        }
        if (own) {
            st4(p.out + base + col, o);
            if (IMG) {
                float4 g2;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float lapt = comp(o, i) - 2.0f * comp(q[M], i) + comp(uo, i);
                    set_comp(g2, i, comp(gr, i) - comp(uf, i) * lapt * p.idt2);
                }
                st4(p.grad + base + col, g2);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) q[j] = q[j + 1];
    }
}

// ---------------------------------------------------------------------------
// 2D step ([x][z]). Block: BZ threads, tile of TZ = 4 BZ z points, streaming x.
// ---------------------------------------------------------------------------
template <int M, int BZ, bool IMG>
__global__ void __launch_bounds__(BZ) k_step2d(const StepParams p) {
    constexpr int TZ = 4 * BZ;
    constexpr int P = (M + 3) & ~3;
    constexpr int HZ = P / 4;
    constexpr int LW = TZ + 2 * P;
    __shared__ __attribute__((aligned(16))) float lds[LW];

    const int r = xcd_remap(blockIdx.x, p.nblocks);
    if (r >= p.nblocks) return;
    const int itz = r % p.ntz;
    const int ich = r / p.ntz;
    const int tid = threadIdx.x;
    const int z0 = itz * TZ;
    const int z = z0 + 4 * tid;
    const bool own = z < p.nz;
    const int xb = ich * p.cx;
    const int xe = min(xb + p.cx, p.nx);
    const int64_t col = own ? z : 0;

    float ez[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ez[i] = (own && z + i < p.nz) ? p.etaz[z + i] : 0.0f;

    float4 q[2 * M + 1];
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) {
        const int xx = xb - M + j;
        q[j] = (own && xx >= 0 && xx < p.nx) ? ld4(p.cur + (int64_t)xx * p.sx + col) : zero4();
    }

    for (int x = xb; x < xe; ++x) {
        const int64_t base = (int64_t)x * p.sx;
        {
            const int xn = x + M;
            q[2 * M] = (own && xn < p.nx) ? ld4(p.cur + (int64_t)xn * p.sx + col) : zero4();
        }
        const float4 uo = own ? ld4(p.old + base + col) : zero4();
        const float4 kp = own ? ld4(p.kap + base + col) : zero4();
        float4 uf = zero4(), gr = zero4();
        if (IMG && own) {
            uf = ld4(p.ufwd + base + col);
            gr = ld4(p.grad + base + col);
        }
        const float ex = p.etax[x];

        st4(lds + P + 4 * tid, q[M]);
        for (int i = tid; i < 2 * HZ; i += BZ) {
            const int side = i / HZ, kk = i - side * HZ;
            const int lc = side ? (P + TZ + 4 * kk) : 4 * kk;
            const int gz = z0 - P + lc;
            float4 v = zero4();
            if (gz >= 0 && gz < p.nz) v = ld4(p.cur + base + gz);
            st4(lds + lc, v);
        }
        __syncthreads();

        float lap[4];
        {
            const float4 c = q[M];
#pragma unroll
            for (int i = 0; i < 4; ++i) lap[i] = p.c0 * comp(c, i);
#pragma unroll
            for (int j = 1; j <= M; ++j) {
                const float4 a = q[M - j], b = q[M + j];
                lap[0] = fmaf(p.wx[j], a.x + b.x, lap[0]);
                lap[1] = fmaf(p.wx[j], a.y + b.y, lap[1]);
                lap[2] = fmaf(p.wx[j], a.z + b.z, lap[2]);
                lap[3] = fmaf(p.wx[j], a.w + b.w, lap[3]);
            }
            float w[2 * P + 4];
#pragma unroll
            for (int k = 0; k < (2 * P + 4) / 4; ++k) {
                const float4 v = ld4(lds + 4 * tid + 4 * k);
                w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 1; j <= M; ++j)
                    lap[i] = fmaf(p.wz[j], w[P + i - j] + w[P + i + j], lap[i]);
        }

        float4 o;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = update(comp(q[M], i), comp(uo, i), comp(kp, i), lap[i], ex + ez[i], p.inv2dt);
            if (z + i >= p.nz) v = 0.0f;
            set_comp(o, i, v);
        }
        if (own) {
            st4(p.out + base + col, o);
            if (IMG) {
                float4 g2;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float lapt = comp(o, i) - 2.0f * comp(q[M], i) + comp(uo, i);
                    set_comp(g2, i, comp(gr, i) - comp(uf, i) * lapt * p.idt2);
                }
                st4(p.grad + base + col, g2);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) q[j] = q[j + 1];
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

__global__ void k_copy(const float* __restrict__ s, float* __restrict__ d, int64_t n) {
    const int64_t n4 = n / 4;
    const float4* s4 = reinterpret_cast<const float4*>(s);
    float4* d4 = reinterpret_cast<float4*>(d);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        d4[i] = s4[i];
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
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

unsigned rows_grid(int nx, int ny) {
    return (unsigned)std::min<int64_t>((int64_t)nx * ny, 65535);
}

int grid_1d(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

template <int M>
hipError_t launch_step_m(const StepParams& p, int ndim, bool img, hipStream_t s) {
    const TileShape ts = step_tile(ndim, M);
    const int grid = ((p.nblocks + 7) / 8) * 8;
    if (ndim == 3) {
        if (ts.bz != 16 || ts.by != 16) return hipErrorInvalidValue;
        if (img) hipLaunchKernelGGL((k_step3d<M, 16, 16, true>), dim3(grid), dim3(256), 0, s, p);
        else hipLaunchKernelGGL((k_step3d<M, 16, 16, false>), dim3(grid), dim3(256), 0, s, p);
    } else {
        if (ts.bz != 64) return hipErrorInvalidValue;
        if (img) hipLaunchKernelGGL((k_step2d<M, 64, true>), dim3(grid), dim3(64), 0, s, p);
        else hipLaunchKernelGGL((k_step2d<M, 64, false>), dim3(grid), dim3(64), 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace

TileShape step_tile(int ndim, int /*half*/) {
    if (ndim == 3) return TileShape{16, 16};
    return TileShape{64, 1};
}

void step_plan(StepParams& p, int ndim, int half, int cx_request) {
    const TileShape ts = step_tile(ndim, half);
    const int tz = 4 * ts.bz;
    p.ntz = (p.nz + tz - 1) / tz;
    p.nty = ndim == 3 ? (p.ny + ts.by - 1) / ts.by : 1;
    const int64_t tiles = (int64_t)p.ntz * p.nty;
    int cx = cx_request;
    if (cx <= 0) {
        // enough blocks to fill 256 CUs several times over, but chunks long
        // enough that the 2M-plane register warm-up stays a small overhead
        const int64_t want = 2048;
        int64_t nch = (want + tiles - 1) / tiles;
        cx = (int)std::max<int64_t>(1, (p.nx + nch - 1) / nch);
        cx = std::max(cx, std::min(p.nx, 6 * half));
    }
    p.cx = std::min(cx, p.nx);
    p.nchunks = (p.nx + p.cx - 1) / p.cx;
    p.nblocks = (int)(tiles * p.nchunks);
}

hipError_t launch_step(const StepParams& p, int ndim, int half, bool imaging, hipStream_t s) {
    if (p.nblocks <= 0) return hipSuccess;
    switch (half) {
        case 2: return launch_step_m<2>(p, ndim, imaging, s);
        case 3: return launch_step_m<3>(p, ndim, imaging, s);
        case 4: return launch_step_m<4>(p, ndim, imaging, s);
        case 5: return launch_step_m<5>(p, ndim, imaging, s);
        case 6: return launch_step_m<6>(p, ndim, imaging, s);
        case 7: return launch_step_m<7>(p, ndim, imaging, s);
        case 8: return launch_step_m<8>(p, ndim, imaging, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inject(const InjectParams& p, hipStream_t s) {
    if (p.nnodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject, dim3((p.nnodes + 255) / 256), dim3(256), 0, s, p);
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

hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(grid_1d(n / 4 + 1, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* x, int64_t n, unsigned int* count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_1d(n, 256)), dim3(256), 0, s, x, n, count);
    return hipGetLastError();
}

hipError_t launch_minmax(const float* x, int64_t n, float* out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minmax, dim3(grid_1d(n, 256)), dim3(256), 0, s, x, n,
                       reinterpret_cast<unsigned int*>(out3));
    return hipGetLastError();
}

}  // namespace wf
