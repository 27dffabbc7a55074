// Internal interface between the host runtime and the gfx950 kernels.
// Everything here is device-side data layout and launch plumbing; the public
// C ABI is include/wavefd.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace wf {

constexpr int kMaxHalf = 8;   // space order up to 16

// Number of zero ghost x-planes kept before and after every field that the
// step kernels read (one update per launch needs M + its prefetch distance,
// at most 10; two updates per launch 2M + its prefetch distance, at most 9
// for the compiled orders, checked at compile time).
constexpr int kGhostPlanes = 12;

// What the step kernel does besides the update (template variants).
enum StepMode : int {
    kModePlain = 0,         // the update only
    kModeImaging = 1,       // grad -= ufwd (out - 2 cur + old) / dt^2   (adjoint sweep of the gradient)
    kModeBornSource = 2,    // grad = -ufwd (out - 2 cur + old), ufwd = dm   (Born source of the next scattered step)
    kModeVolumeSource = 3,  // kap vsrc / dt^2 added inside the update   (a source on every node)
    kModeCount = 4
};

// Parameters of one time step of the fused update
//   out = (2 cur - (1 - g) old + kap * Lap(cur)) / (1 + g),  g = eta kap / (2 dt)
// on a pitched field layout: element (x, y, z) at x*sx + y*sy + z, sy = pitch
// (a multiple of 4 floats, >= nz rounded up to 4; the pad is kept at zero).
// cur, old, kap, ufwd and grad point at plane 0 of allocations that extend by
// kGhostPlanes zero planes on both sides in x.
// `out` may alias `old` (in-place update; every element of old is read by the
// thread that then writes the same element of out).
// With imaging on (adjoint sweeps of the gradient): grad -= ufwd * (out - 2 cur
// + old) / dt^2, using `out` before any receiver injection (whose part the
// injecting thread subtracts itself). Born source: grad = -ufwd * (out - 2 cur +
// old) with out after injection. Volume source: the numerator of the update
// gets kap * vsrc / dt^2, i.e. out += (dt^2 / a) * vsrc / dt^2 * dt^2.
struct StepParams {
    const float* cur;
    const float* old;
    float* out;
    const float* kap;
    const float* etax;   // per-axis damping profiles (eta = etax + etay + etaz)
    const float* etay;   // unused in 2D
    const float* etaz;
    float* grad;
    const float* ufwd;
    const float* vsrc;   // volume source (kModeVolumeSource), pitched like the fields
    int nx, ny, nz;      // ny == 1 in 2D
    int64_t sx, sy;      // strides in floats
    int cx;              // x-chunk length per block
    int ntz, nty, nchunks, nblocks;
    float c0;            // alpha_0 * sum_a 1/h_a^2
    float wx[kMaxHalf + 1], wy[kMaxHalf + 1], wz[kMaxHalf + 1];  // alpha_j / h_a^2
    float inv2dt;
    float idt2;
    int tile;            // host side: which compiled tile shape step_plan chose

    // Fused sampling of `cur`: block r (tile index) writes, for i in
    // [r smp_per, (r + 1) smp_per), smp_out[i] = sum_k smp_w[i*K+k] cur[smp_off[i*K+k]]
    // with K = 2^D corners per point.
    const int64_t* smp_off;
    const float* smp_w;
    float* smp_out;      // NULL: no sampling
    int smp_n, smp_per;

    // Fused injection into `out`: entries grouped by block (inj_blk, nblocks+1
    // offsets), inside a block by (thread, x); an entry is one (thread, plane)
    // pair with the increments of its 4 z nodes (zero where no node), and
    // thread t of block b owns the entry range inj_thr[b*NT + t]. inj_inc
    // holds this step's increments, one float4 per entry.
    const int* inj_blk;  // NULL: no injection
    const int2* inj_thr;
    const int* inj_x;
    const float4* inj_inc;
};

// Largest number of injection entries a block can stage in LDS (20 bytes
// each): 3D blocks span 8 rows and hold many receivers; 2D blocks are one row
// and small, so that their LDS does not limit residency.
constexpr int kInjCap3 = 1024;
constexpr int kInjCap2 = 256;
inline int inj_cap(int ndim) { return ndim == 3 ? kInjCap3 : kInjCap2; }

// One grid of a batched step launch (see k_step_batch).
struct BatchJob {
    StepParams p;          // planned for this grid; cur/old/out set per step
    float* buf0;           // u^{n0} at the first step of the launch sequence
    float* buf1;           // u^{n0-1}
    int64_t inj_stride;    // floats per row of the injection increments
    int64_t smp_stride;    // floats per row of the sampled record
    int n0;                // step index at k = 0
    int nsteps;            // steps of this grid in the sequence
    int block_begin;       // first block (a multiple of 8)
    int nblk;              // blocks of this grid (sampling + stencil)
};

// Launch step k of a batch sequence over njobs grids of dimension ndim and
// half order `half`, all planned with the same tile shape; total_blocks is the
// end of the last job's block range.
hipError_t launch_step_batch(const BatchJob* jobs_dev, int njobs, int total_blocks, int ndim,
                             int half, int tile, int k, hipStream_t s);

// Forward shots of grids small enough that both wavefields fit one
// work-group's LDS (the serving engine's resident teams): each work-group of
// a launch takes a shot from the launch's table, steps it to the end with
// only work-group barriers (the fields never leave LDS), writes its record and
// takes the next; or, for few shots, each shot split over a team of W
// work-groups that recompute their neighbours' nearest planes for `period`
// updates and then exchange boundary planes through global memory with one
// barrier. The source increments are made beforehand by launch_increments
// over the point set's node tables. Results equal wf_forward's bit for bit
// (the same arithmetic in the same order).
constexpr int kTeamThreads = 1024;
constexpr int kTeamFieldFloats = 40640;   // two fields of nx * ny * round4(nz) floats
struct TeamJob {
    int ndim, half, nx, ny, nz, nt, nrec, nnodes;
    float c0, inv2dt;
    float wx[kMaxHalf + 1], wy[kMaxHalf + 1], wz[kMaxHalf + 1];
    int64_t sx, sy;             // the model's pitched layout (offsets of kap and of the point tables)
    const float* kap;
    const float* etax;
    const float* etay;
    const float* etaz;
    const int64_t* noff;        // source nodes (pitched offsets)
    const float* inc;           // [nt-1][nnodes] their increments per step (k_increments)
    const int64_t* smp_off;     // receiver corners (pitched offsets) and weights [nrec][2^ndim]
    const float* smp_w;
    float* rec;                 // [nt][nrec]
};
struct TeamArgs {
    const TeamJob* jobs;        // device memory, njobs shots of one (ndim, half)
    unsigned int* next;         // device memory, 0 at the launch (width 1)
    int njobs;
    int width;                  // work-groups per shot: 1, or W > 1 (the launch is teams x W work-groups)
    int period;                 // width > 1: updates between exchanges (every part owns >= period M planes)
    float4* exch;               // width > 1: boundary planes, exch_stride float4 per shot
    int64_t exch_stride;        //   (2 x W x 2 x 2 x period M planes of the shot's plane size)
    unsigned int* cnt;          // width > 1: one barrier counter per shot, 32 apart, 0 at the launch
    unsigned int* err;          // 0 at the launch; nonzero after it: a barrier wait timed out
    unsigned long long limit;   // longest barrier wait (s_memrealtime ticks, 100 MHz)
};
// A grid fits a team when both fields (z padded to 4) fit kTeamFieldFloats.
bool team_fits(int64_t nx, int64_t ny, int64_t nz);
hipError_t launch_team(const TeamArgs& a, int ndim, int half, int nwg, hipStream_t s);

// Two plain updates in one pass (2D and 3D, half orders 2 and 4): u^{n+1}
// and u^{n+2} from u^n and u^{n-1}, each node with the arithmetic of the
// single-update kernel (so the fields are the same bits). A block owns an
// inner (y, z) tile of by x 4(step2_cols - 2 hz) nodes (hz = ceil(M / 4); in
// 3D by = 20 at half order 2 and 16 at 4, in 2D one row) and an x chunk; it
// computes u^{n+1} on the tile extended by M rows (3D) and 4 hz nodes on
// each side and on M planes beyond either end of its chunk, keeps it in
// registers and LDS, and from it u^{n+2} on the inner tile. Reads u^n,
// u^{n-1} and kap, writes u^{n+1} and u^{n+2} (20 bytes per node for two
// updates). None of the four fields may alias another: neighbouring blocks
// read cur and old where this block writes.
// float4 columns per row of the extended tile, and injection entries per
// block and update (a 2D block is one row and stages fewer, so that several
// blocks fit a CU's LDS)
__host__ __device__ constexpr int step2_cols(bool d3) { return d3 ? 32 : 128; }
__host__ __device__ constexpr int step2_inj_cap(bool d3) { return d3 ? 512 : 128; }
struct Step2Params {
    const float* cur;    // u^n
    const float* old;    // u^{n-1}
    float* out1;         // u^{n+1}
    float* out2;         // u^{n+2}
    const float* kap;
    const float* etax;
    const float* etay;
    const float* etaz;
    int nx, ny, nz;
    int64_t sx, sy;
    int cx;              // x-chunk length per block
    int ntz, nty, nchunks, nblocks;
    int by;              // host side: the compiled tile height the planner chose
    float c0;
    float wx[kMaxHalf + 1], wy[kMaxHalf + 1], wz[kMaxHalf + 1];
    float inv2dt;
    // receivers: block r samples points [r smp_per, (r + 1) smp_per) of cur
    // into smp_cur and of old into smp_old (either may be NULL)
    const int64_t* smp_off;
    const float* smp_w;
    float* smp_cur;
    float* smp_old;
    int smp_n, smp_per;
    // injection, as in StepParams, for the first update ([0]: entries over
    // the extended tile and chunk, increments of step n) and the second ([1]:
    // the inner tile and chunk, step n + 1); inj_blk[k] NULL: none
    const int* inj_blk[2];
    const int2* inj_thr[2];
    const int* inj_x[2];
    const float4* inj_inc[2];
};
// Whether the two-update kernel is compiled for (ndim, half), and whether
// it was measured faster than two single-update launches on a grid of that
// many nodes.
bool step2_supported(int ndim, int half);
bool step2_preferred(int ndim, int half, int64_t nodes);
// Plan tiles and chunks from the grid in p (nx, ny, nz set); cx_request > 0
// forces the chunk length.
void step2_plan(Step2Params& p, int ndim, int half, int cx_request);
// Threads per block of the planned launch, and the extension in float4
// columns on each side of the inner tile (the extension in rows is half in
// 3D, none in 2D).
int step2_threads(int ndim, int half, int by);
int step2_ext_cols(int half);
hipError_t launch_step2(const Step2Params& p, int ndim, int half, hipStream_t s);

// Tile shapes (threads along z carry 4 points each).
struct TileShape {
    int bz, by;   // threads along z and y per block
};

TileShape step_tile(int ndim, int tile);
// Choose the tile shape and the x-chunking (ntz/nty/nchunks/nblocks/cx); a
// positive cx_request forces the chunk length, tile_request >= 0 the shape.
void step_plan(StepParams& p, int ndim, int half, int mode, int cx_request, int tile_request);
hipError_t launch_step(const StepParams& p, int ndim, int half, int mode, hipStream_t s);

// Sparse injection at unique nodes (deterministic, no atomics):
//   field[off[i]] += scale_i * sum_{e in seg i} w[e] * vals[pt[e]],
//   scale_i = kap / (1 + eta_i kap / (2 dt)) at that node;
// with imaging: grad[off[i]] -= ufwd[off[i]] * that increment / dt^2.
struct InjectParams {
    float* field;
    const float* kap;
    const int64_t* off;
    const float* eta;
    const int* seg;      // nnodes + 1 offsets into pt/w
    const int* pt;
    const float* w;
    const float* vals;   // one row of the [nt][npts] series
    float* grad;
    const float* ufwd;
    const float* vsrc;   // volume source (kModeVolumeSource), pitched like the fields
    int nnodes;
    float inv2dt, idt2;
};
hipError_t launch_inject(const InjectParams& p, hipStream_t s);

// Increments of the fused injection for every step:
//   inc[n * nnodes + k] = (sum_{e in seg k} w[e] vals[n * npts + pt[e]]) * kap/(1 + eta kap/(2 dt))
// at node k (pitched offset off[k], damping eta[k]), n = 0..nrows-1.
struct IncParams {
    float* inc;
    const float* kap;
    const int64_t* off;
    const float* eta;
    const int* seg;
    const int* pt;
    const float* w;
    const float* vals;
    int nnodes, npts, nrows;
    float inv2dt;
};
hipError_t launch_increments(const IncParams& p, hipStream_t s);

// out[i] = sum_k w[i*K + k] * field[off[i*K + k]]
hipError_t launch_sample(const float* field, const int64_t* off, const float* w, int npts,
                         int K, float* out, hipStream_t s);

// kap (pitched) = dt^2 / m (dense), computed in FP64; pad set to zero.
hipError_t launch_coef(const float* m_dense, float* kap, int nx, int ny, int nz, int64_t sx,
                       int64_t sy, double dt, hipStream_t s);
// pitched -> dense and dense -> pitched copies (pad of the pitched side zeroed).
hipError_t launch_unpitch(const float* src, float* dst, int nx, int ny, int nz, int64_t sx,
                          int64_t sy, hipStream_t s);
hipError_t launch_pitch(const float* src, float* dst, int nx, int ny, int nz, int64_t sx,
                        int64_t sy, hipStream_t s);
hipError_t launch_fill(float* dst, int64_t n, float v, hipStream_t s);
// count of non-finite values in x[0..n) added to *count
hipError_t launch_count_nonfinite(const float* x, int64_t n, unsigned int* count, hipStream_t s);
// r = d - d_obs (r may alias d); partial[b] = sum over block b of r^2 in FP64,
// for nblocks = residual_blocks(n) blocks (summed on the host in fixed order).
int residual_blocks(int64_t n);
hipError_t launch_residual(const float* d, const float* d_obs, float* r, int64_t n, double* partial,
                           hipStream_t s);
// Face slabs just outside an interior box: along each axis a slab M nodes
// deep on either side, spanning the box along the other axes (clipped to the
// grid). Their union holds every node outside the box that the order-2M
// stencil of a box node reads.
struct StripGeom {
    int nslab = 0;
    int64_t start[7] = {0, 0, 0, 0, 0, 0, 0};   // prefix counts of the slabs
    int x0[6], x1[6], y0[6], y1[6], z0[6], z1[6];
    int64_t sx = 0, sy = 0;
};
// to_field = 0: strip[i] = field[node i]; 1: field[node i] = strip[i]
hipError_t launch_strip(float* field, float* strip, const StripGeom& g, int to_field, hipStream_t s);
// zero every node of a pitched field outside [bx0,bx1) x [by0,by1) x [bz0,bz1)
hipError_t launch_mask_box(float* field, int nx, int ny, int nz, int64_t sx, int64_t sy, int bx0,
                           int bx1, int by0, int by1, int bz0, int bz1, hipStream_t s);
// m[i] = min(max(m[i] - alpha g[i], lo), hi) (one rounding: fma)
hipError_t launch_update(float* m, const float* g, float alpha, float lo, float hi, int64_t n,
                         hipStream_t s);
// min and max of m over n values into out[0], out[1] (out pre-filled by caller)
hipError_t launch_minmax(const float* x, int64_t n, float* out2, hipStream_t s);

}  // namespace wf
