/*
 * wavefd.h - C ABI of an MI355X (gfx950) explicit finite-difference acoustic
 * propagator: forward modelling, its exact discrete adjoint, the adjoint-state
 * gradient with optimal checkpointing or boundary-wavefield reconstruction,
 * the multi-shot FWI gradient and fixed-step update, linearised (Born)
 * modelling, and a continuous-batching serving engine.
 *
 * The operations follow arxiv 1808.01995 (Louboutin et al., Devito v3.1.0):
 *   - PDE: m u_tt - Lap u + eta u_t = q, m = 1/c^2 the squared slowness
 *     (eq. acoustic, eq. fdWE-abc, Section "Boundary conditions");
 *   - space: centred second differences of even order k = space_order per axis
 *     (eq. fdSpace), summed into the Laplacian;
 *   - time: second-order centred difference (eq. fdTime), explicit update
 *     (eq. eulerfwd) with the damping term differenced centrally:
 *         a u^{n+1} = 2 m u^n - b u^{n-1} + dt^2 Lap u^n,
 *         a = m + eta dt/2, b = m - eta dt/2;
 *   - zero Dirichlet values beyond the computational grid (Section "Acoustic
 *     forward modelling operator");
 *   - sources injected and receivers interpolated multilinearly inside the
 *     containing cell (Section "Sparse point interpolation"); a source sample
 *     q^n enters u^{n+1} with weight dt^2/a (dt^2/m where eta = 0);
 *   - adjoint: the transpose A(m)^T, i.e. backward substitution (matrix view in
 *     Section "Temporal discretization"; eq. Adj);
 *   - gradient of Phi = 1/2 ||P_r u - d||^2 (eqs. AS, Grad):
 *         g = - sum_{j=1}^{nt-1} u^j (v^{j-1} - 2 v^j + v^{j+1}) / dt^2,
 *     with the forward wavefield kept by optimal (revolve) checkpointing or
 *     rebuilt from stored boundary values (Section "Discrete adjoint
 *     wave-equation and FWI gradient");
 *   - FWI: the objective and gradient summed over source experiments and a
 *     fixed-step update (Section "FWI using Devito operators");
 *   - J dm, the Jacobian of eq. Grad applied to a model perturbation.
 *
 * Conventions shared by every call:
 *   - Physical grid n[0..ndim-1] nodes with spacing h (m); a damping layer of
 *     nbl nodes is added outside it on every side, so the computational grid
 *     has Nc_a = n_a + 2 nbl nodes. Arrays on the computational grid are dense,
 *     C-order [x][y][z] (3D) or [x][z] (2D), z contiguous, FP32.
 *   - Units: metres, milliseconds, km/s; m in (ms/m)^2.
 *   - Coordinates are FP64 metres relative to the physical origin, in the
 *     order (x, z) or (x, y, z); a point must lie inside the computational grid
 *     (-nbl h_a <= x_a - origin_a <= (n_a - 1 + nbl) h_a), else WF_E_DOMAIN.
 *   - Time axis: nt samples t_n = n dt (nt - 1 updates). Wavelets and records
 *     are [nt][npoints] row-major FP32 device arrays. Record row 0 is P_r u^0 = 0.
 *   - Damping: eta = sum_a eta_max_a (d_a/nbl)^p, d_a = distance (nodes) from
 *     the physical grid along axis a, eta_max_a = 3 ln(1/R) / (2 nbl h_a c_ref).
 *
 * Ownership: the caller owns every pointer it passes (device buffers and host
 * coordinate arrays); host arrays are read before the call returns, device
 * inputs are read by work enqueued on `stream` and outputs are written in
 * stream order. The library owns only what its handles hold (wavefields,
 * coefficients, checkpoints, sparse tables), freed by the matching destroy.
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL means the default
 * stream. Calls enqueue work and return without synchronising, except where
 * noted. A model used on one stream and then on another orders the new
 * stream's work after the old one's (an event, no host wait), so calls in
 * turn on different streams need no synchronisation between them. A handle is
 * not thread-safe: use one per host thread.
 *
 * Errors: every call returns a wf_status. Argument, shape, CFL, domain and
 * budget errors are detected on the host before anything is enqueued and leave
 * no side effect. wf_last_error() returns a message for the calling thread's
 * most recent failure. No C++ exception crosses this interface.
 */
#ifndef WAVEFD_H
#define WAVEFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int wf_status;

#define WF_OK            0
#define WF_E_ARG        -1  /* bad argument, shape or order                  */
#define WF_E_DOMAIN     -2  /* a sparse point lies outside the grid           */
#define WF_E_CFL        -3  /* dt above the stability limit wf_critical_dt()  */
#define WF_E_NOMEM      -4  /* device allocation failed                       */
#define WF_E_BUDGET     -5  /* the request does not fit the HBM budget        */
#define WF_E_HIP        -6  /* a HIP runtime call failed                      */
#define WF_E_NONFINITE  -7  /* a non-finite value was produced (validation)   */
#define WF_E_STATE      -8  /* handle in the wrong state / unknown ticket     */

typedef struct {
    int     ndim;         /* 2 or 3                                              */
    int64_t n[3];         /* physical nodes per axis (x, [y,] z)                 */
    double  h[3];         /* spacing per axis (m)                                */
    double  origin[3];    /* physical origin (m)                                 */
    int     nbl;          /* damping-layer width in nodes (>= 0)                 */
    int     space_order;  /* k: even, 4..16                                      */
    double  c_ref;        /* damping reference velocity (km/s), > 0              */
    double  R;            /* nominal reflection coefficient; 0 selects 1e-3      */
    int     eta_power;    /* damping profile power p (1..4); 0 selects 2         */
} wf_geom;

typedef struct wf_model  wf_model;   /* opaque, device-resident model          */
typedef struct wf_engine wf_engine;  /* opaque serving engine                  */

/* Message for the calling thread's last failure ("" if none). The pointer stays
 * valid until the next call on the same thread. */
const char* wf_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int wf_version(void);

/* Stability limit of the explicit update (eq. eulerfwd) for this geometry:
 * dt_crit = 2 / (vmax sqrt(S sum_a h_a^-2)), S = sum of |weights| of the order-k
 * 1D stencil. Pure host function; returns a negative value on bad input. */
double wf_critical_dt(const wf_geom* geom, double vmax);

/* Computational-grid shape of `geom` (Nc per axis, 1 for unused axes) and the
 * number of computational nodes. Pure host function. */
wf_status wf_geom_shape(const wf_geom* geom, int64_t shape_out[3], int64_t* npoints_out);

/* Create a device-resident model from the squared slowness m on the
 * computational grid (dense FP32, Nc^D, device pointer, all values > 0 and
 * finite). The library copies what it needs; m_dev may be freed after the work
 * enqueued on `stream` has run. */
wf_status wf_model_create(const wf_geom* geom, const float* m_dev, void* stream,
                          wf_model** out);

/* Replace the model's squared slowness (same layout as in create). */
wf_status wf_model_set_m(wf_model* model, const float* m_dev, void* stream);

/* Device bytes held by the model handle itself (fields, coefficients, sparse
 * tables, and the gradient workspace: the checkpoint pool of the last
 * gradient call is kept for the next one, because allocating tens of GB of
 * device memory again costs seconds). */
int64_t wf_model_bytes(const wf_model* model);

/* Free the model's cached gradient workspace and the second pair of
 * wavefields of the two-update forward loop; the next call that needs them
 * allocates them again. Synchronises the model's device work. */
wf_status wf_model_trim(wf_model* model);

/* Validation aid. Outside the computational grid the wavefield is zero
 * (Section "Boundary conditions": the zero Dirichlet condition beyond the
 * damping layer); the library stores that outside as ghost planes before and
 * after the x range and as row padding beyond nz of every pitched field, which
 * the stencil reads and no kernel may write. Stores in *count the number of
 * nonzero values (NaN included) found there in the model's kappa and
 * wavefield buffers and, while it is marked clean, in every field slot of its
 * gradient workspace (after a boundary-reconstruction gradient it is not: its
 * slabs reuse those slots until the next gradient call clears them). 0 after
 * any correct sequence of calls. Waits for the model's device work; blocks;
 * allocates 8 bytes of device memory. NULL arguments: WF_E_ARG. */
wf_status wf_model_ghost_nonzero(wf_model* model, int64_t* count);

/* Time loops of wf_forward / wf_adjoint on this model that were launched as a
 * captured HIP graph. While capture is enabled (wf_graph_enable), a call runs
 * eagerly the first time its signature (dt, nt, point coordinates, every
 * device pointer, save_every) is seen; when the same signature comes back
 * within the next few calls, that call captures the whole loop on the model's
 * own stream and launches it, and later calls with it replay the graph (up to
 * four captured loops are kept per model, least recently used dropped first).
 * Graph launches are ordered after earlier work on the caller's stream and
 * before later work on it. The contents of the inputs (m, wavelets, data) may
 * change between calls; only pointers and sizes are part of the signature.
 * Kernel timing (wf_profile_enable) suspends capture. Returns -1 for a NULL
 * model. */
int64_t wf_model_graph_launches(const wf_model* model);

/* Process-wide switch of the post-run validation: 1 on, 0 off; off by default,
 * on at start-up when the environment sets WAVEFD_VALIDATE=1. The paper's
 * scheme is stable only under its time-step condition (Section "Temporal
 * discretization"), which every call enforces before any work; non-finite
 * inputs (a wavelet, residual, dm or m holding Inf or NaN) still propagate.
 * While on, wf_forward (rec_out, u_save), wf_adjoint (src_out), wf_gradient
 * (grad_out), wf_born (drec_out, rec_out) and wf_fwi_gradient (grad_out, each
 * d_pred, the misfit) count the non-finite values of their outputs after the
 * run, waiting for the stream, and return WF_E_NONFINITE if there are any
 * (the outputs are written all the same). Requests served by the engine are
 * not checked. */
wf_status wf_validate_enable(int on);

/* Process-wide switch for that capture: 1 on, 0 off. Off by default (a
 * replayed kernel node was measured slower than a stream launch on ROCm 7.x),
 * on at start-up when the environment sets WAVEFD_GRAPH=1. Captured loops are
 * kept while it is off and used again once it is switched back on. */
wf_status wf_graph_enable(int on);

/* Process-wide mode for running the time loops of wf_forward and wf_adjoint
 * on models of space order 4 or 8 two updates (eq. eulerfwd with the damping
 * of eq. fdWE-abc, applied twice) per kernel launch: the launch reads u^n,
 * u^{n-1} and kappa once and writes u^{n+1} and u^{n+2}, 20 bytes per node
 * for two updates instead of 32 (the update is bound by memory traffic,
 * Section "Performance"), at the price of recomputing u^{n+1} on a margin
 * around every tile (M rows in 3D, 4 nodes along z in 2D and 3D). 0: one
 * update per launch; 1 (the default): two where that was measured faster
 * (2D order 4 at every size, 2D order 8 from 5e7 nodes, 3D order 4 from 9e7
 * nodes); 2: two wherever compiled (orders 4 and 8, 2D and 3D). The
 * environment's WAVEFD_TWO_STEP=0 or =2 sets the mode at start-up. Records,
 * saved fields and the final fields are the same bits in every mode. Such a
 * loop keeps a second pair of wavefields in the model (counted by
 * wf_model_bytes, freed by wf_model_trim); calls made through the serving
 * engine or the allocation-free entry point keep one update per launch, and
 * so does a loop whose sources crowd a block beyond what it can stage or for
 * which those two fields cannot be allocated. Other modes: WF_E_ARG. */
wf_status wf_two_step_enable(int mode);

/* Free the model and everything it holds. Synchronises its device work. */
wf_status wf_model_destroy(wf_model* model);

/* Forward modelling d = P_r A(m)^{-1} P_s^T q (Section "Acoustic forward
 * modelling operator").
 *   src_xyz  host FP64 [nsrc][ndim];  src_wav device FP32 [nt][nsrc]
 *   rec_xyz  host FP64 [nrec][ndim];  rec_out device FP32 [nt][nrec] (written)
 *   u_save   device FP32 [(nt-1)/save_every + 1][Nc^D] or NULL: receives u^n
 *            for n = 0, save_every, 2 save_every, ... (dense layout)
 * nt >= 1, nsrc >= 0, nrec >= 0, 0 < dt <= wf_critical_dt(geom, vmax(m)). */
wf_status wf_forward(wf_model* model, double dt, int nt,
                     int nsrc, const double* src_xyz, const float* src_wav,
                     int nrec, const double* rec_xyz, float* rec_out,
                     float* u_save, int save_every, void* stream);

/* wf_forward for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid allocation while they run): the same
 * modelling with u_save = NULL, the same kernels and the same bits, but the
 * call's sparse-point tables, fused injection tables and per-step injection
 * increments are carved from a fixed 32 MiB device scratch that the library
 * holds per GPU until the process ends, instead of the model's cached
 * allocations. It calls no device allocation or free. Limits: the tables of
 * nsrc + nrec points plus nt rows of 4 x (nodes touched by the sources)
 * floats must fit the 32 MiB (about nt x nsrc x 2^D x 16 bytes for the
 * increments), else WF_E_BUDGET before any work is queued. The call first
 * waits for `stream` (earlier calls on it may still read the scratch) and
 * blocks while it uploads the tables; it is not graph-capturable for that
 * reason. Calls that overlap on one GPU (on different streams or threads)
 * share the scratch and race: serialise them. The model itself, created by
 * wf_model_create, holds the fields and coefficients. */
wf_status wf_forward_noalloc(wf_model* model, double dt, int nt,
                             int nsrc, const double* src_xyz, const float* src_wav,
                             int nrec, const double* rec_xyz, float* rec_out, void* stream);

/* Adjoint x = P_s A(m)^{-T} P_r^T y (eq. Adj): the exact transpose of
 * wf_forward with the same arguments. rec_in device FP32 [nt][nrec] (row 0 is
 * never used), src_out device FP32 [nt][nsrc] (written; row nt-1 is 0). */
wf_status wf_adjoint(wf_model* model, double dt, int nt,
                     int nrec, const double* rec_xyz, const float* rec_in,
                     int nsrc, const double* src_xyz, float* src_out, void* stream);

/* Adjoint-state gradient (eqs. Grad, Adj) of Phi = 1/2 ||P_r u - d_obs||^2 at
 * the model's m for the given residual r = P_r u - d_obs (device FP32
 * [nt][nrec]); grad_out device FP32 Nc^D (dense, overwritten).
 *   n_checkpoints  > 0: revolve with that many stored states (2 fields each);
 *                  -1 : store every forward wavefield (no recomputation);
 *                   0 : the largest count that fits hbm_budget_bytes;
 *                  -2 : boundary-wavefield reconstruction (the alternative
 *                       to checkpointing in Section "Discrete adjoint
 *                       wave-equation and FWI gradient"): the forward sweep
 *                       stores per step only the M-deep face slabs around
 *                       the physical grid, and u is rebuilt backward on the
 *                       physical grid during the adjoint sweep (one extra
 *                       wave solve, memory 4 fields + nt x slabs). The
 *                       damping layer cannot be rebuilt backward, so
 *                       grad_out is the gradient on the physical grid and 0
 *                       in the layer.
 *   hbm_budget_bytes  bound on the device memory the call may allocate for
 *                  checkpoints and its temporaries (0: no bound).
 * Results are bitwise identical for every count >= -1; mode -2 agrees with
 * them on the physical grid to FP32 rounding of the backward rebuild.
 * The checkpoint pool is kept by the model for its next gradient call. */
wf_status wf_gradient(wf_model* model, double dt, int nt,
                      int nsrc, const double* src_xyz, const float* src_wav,
                      int nrec, const double* rec_xyz, const float* residual,
                      float* grad_out, int n_checkpoints, int64_t hbm_budget_bytes,
                      void* stream);

/* One source experiment of a multi-shot inversion.
 *   src_xyz host FP64 [nsrc][ndim];  src_wav device FP32 [nt][nsrc]
 *   rec_xyz host FP64 [nrec][ndim];  d_obs   device FP32 [nt][nrec]
 *   d_pred  device FP32 [nt][nrec] or NULL: receives P_r u at the current m */
typedef struct {
    int nsrc;
    const double* src_xyz;
    const float* src_wav;
    int nrec;
    const double* rec_xyz;
    const float* d_obs;
    float* d_pred;
} wf_shot;

/* Multi-shot FWI objective and gradient (Section "FWI using Devito
 * operators": a loop over the source experiments whose gradients are summed;
 * eq. AS per shot). For every shot s, d_s = P_r A(m)^{-1} P_s^T q_s and
 * r_s = d_s - d_obs,s;
 *   misfit_out (host, may be NULL) = 1/2 sum_s ||r_s||^2 (FP64 partial sums
 *              added in a fixed order),
 *   grad_out   (device FP32 Nc^D, dense, overwritten) = sum_s J_s^T r_s.
 * Each shot costs two wave solves: the residual is formed from the record of
 * the gradient's own first forward sweep (plus the recomputation of revolve).
 * n_checkpoints and hbm_budget_bytes apply to each shot as in wf_gradient
 * (the accumulator and the record scratch count against the budget).
 * nshots >= 1; synchronises `stream` (the misfit is a host value). */
wf_status wf_fwi_gradient(wf_model* model, double dt, int nt, int nshots, const wf_shot* shots,
                          float* grad_out, double* misfit_out, int n_checkpoints,
                          int64_t hbm_budget_bytes, void* stream);

/* Fixed-step gradient update of the model's squared slowness (the step of
 * Section "FWI using Devito operators"), projected on bounds:
 *   m <- min(max(m - alpha grad, m_lo), m_hi)  elementwise (one FP32 fma),
 * grad device FP32 Nc^D (dense; every value finite, else WF_E_NONFINITE and m
 * is unchanged), 0 < m_lo <= m_hi (1/vmax^2 and 1/vmin^2; m_hi may be +inf).
 * m_out (device FP32 Nc^D or NULL) receives the new m. The coefficients are
 * recomputed at the next call, whose dt is checked against the new vmax.
 * Synchronises `stream`. */
wf_status wf_model_update(wf_model* model, const float* grad, double alpha, double m_lo,
                          double m_hi, float* m_out, void* stream);

/* Linearised (Born) modelling dd = J dm, J the Jacobian of the forward map
 * m -> P_r u(m) (the operator whose transpose the gradient applies, eq. Grad):
 * the scattered field du solves the update of wf_forward driven by the
 * source -dm (u^{n+1} - 2 u^n + u^{n-1}) / dt^2 (injected with weight dt^2/a
 * on every node), du^0 = 0, dd^n = P_r du^n.
 *   dm       device FP32 Nc^D (dense): squared-slowness perturbation
 *   drec_out device FP32 [nt][nrec] (written)
 *   rec_out  device FP32 [nt][nrec] or NULL: the background record P_r u
 * Other arguments as in wf_forward. wf_gradient with residual r applies the
 * exact transpose: <J dm, r> = <dm, J^T r> to rounding. With the observed
 * data as the residual, wf_gradient gives the reverse-time-migration image
 * J^T d. Synchronises `stream` (it frees its scratch fields). */
wf_status wf_born(wf_model* model, double dt, int nt,
                  int nsrc, const double* src_xyz, const float* src_wav, const float* dm,
                  int nrec, const double* rec_xyz, float* drec_out, float* rec_out, void* stream);

/* Optimal forward-step count of revolve checkpointing (Section "Discrete
 * adjoint wave-equation and FWI gradient"): for `steps` updates to reverse
 * with `snaps` stored states (steps >= 1, snaps >= 1), the closed form
 * r l - C(s + r, r - 1) of Griewank and Walther, r the smallest integer with
 * C(s + r, s) >= l. Pure host function; -1 on bad input. wf_revolve_schedule
 * gives the schedule wf_gradient actually runs. */
int64_t wf_revolve_forward_steps(int64_t steps, int snaps);

#define WF_REVOLVE_ADVANCE  0   /* forward from state `at` to state `arg`       */
#define WF_REVOLVE_TAKESHOT 1   /* store the current state `at` in slot `arg`   */
#define WF_REVOLVE_RESTORE  2   /* make slot `arg` (holding state `at`) current */
#define WF_REVOLVE_REVERSE  3   /* adjoint of step `at` (needs state `at`)      */
#define WF_REVOLVE_FREE     4   /* release slot `arg`                           */

/* The checkpoint schedule that wf_gradient runs with n_checkpoints = snaps
 * (same section): the actions in order, state i being the pair
 * (u^{i+1}, u^i) after i + 1 forward updates, slot 0 holding state 0 from the
 * start. Writes min(count, cap) actions into kind/at/arg (host arrays, may be
 * NULL when cap is 0) and returns the total count, or a negative wf_status
 * for steps < 1 or snaps < 1. Pure host function. */
int64_t wf_revolve_schedule(int64_t steps, int snaps, int32_t* kind, int64_t* at, int64_t* arg,
                            int64_t cap);

/* ------------------------------------------------------------------------ */
/* Kernel timing (tracing aid).                                               */
/* ------------------------------------------------------------------------ */

#define WF_KERNEL_STEP    0   /* the fused time-step kernel                   */
#define WF_KERNEL_INJECT  1   /* sparse injection                              */
#define WF_KERNEL_SAMPLE  2   /* sparse interpolation                          */
#define WF_KERNEL_STEP_RUN 3  /* the whole run of step launches of a forward
                                 or adjoint time loop (wf_profile_runs_enable) */
#define WF_KERNEL_STEP2   4   /* the two-update kernel (wf_two_step_enable)    */
#define WF_KERNEL_STEP2_RUN 5 /* the run of two-update launches of a forward
                                 or adjoint time loop (wf_profile_runs_enable) */

/* While enabled (process-wide), launches of the kernels WF_KERNEL_STEP,
 * WF_KERNEL_INJECT, WF_KERNEL_SAMPLE and WF_KERNEL_STEP2 are
 * bracketed by a pair of HIP events recorded on the stream they run on:
 * every launch for on == 1, every on-th launch of each kind for on > 1 (a
 * lighter touch on the timed work), none for on == 0. */
wf_status wf_profile_enable(int on);

/* While on (process-wide, off by default), every wf_forward and wf_adjoint
 * time loop records one event before its first step launch and one after its
 * last, on the stream they run on: read as kind WF_KERNEL_STEP_RUN, whose
 * launch count is the number of step launches those spans cover, so that the
 * summed time over the count is the average duration of one step launch
 * (gaps between the back-to-back launches included) with two events per
 * loop. A loop that runs two updates per launch records its run of
 * two-update launches as kind WF_KERNEL_STEP2_RUN the same way (and any
 * single update left over as WF_KERNEL_STEP_RUN). Like per-launch timing, it
 * suspends graph capture. */
wf_status wf_profile_runs_enable(int on);

/* Synchronise on the recorded events and return, for kernel `kind`, the summed
 * device time in ms and the number of launches since the last reset; reset != 0
 * clears the record of every kind. */
wf_status wf_profile_read(int kind, double* total_ms, int64_t* launches, int reset);

/* Number of step-kernel launches made since the last reset in kernel mode
 * `mode`: 0 the plain update (forward and adjoint steps, the gradient's
 * forward and recomputed steps), 1 the update with imaging (the gradient's
 * reverse steps), 2 the Born background step, 3 the Born scattered step, 4
 * the two-update launches of forward and adjoint loops (each advancing two
 * plain updates).
 * Counted on the host for every launch, whether timing is on or not; reset
 * != 0 clears every mode after reading. Batched launches of the serving
 * engine are not counted. */
wf_status wf_profile_step_launches(int mode, int64_t* count, int reset);

/* Bandwidth reference for the roofline (Section "Performance", subsection
 * "Roofline analysis", bounds its kernels by a measured stream bandwidth):
 * reads three device arrays of n_floats floats and writes a fourth - the
 * step kernel's 16 bytes per node with no stencil, halo or reuse - one float4
 * per thread with non-temporal loads and stores, once to warm up and then
 * `reps` times on a stream of its own, and stores in *gbs_out the rate in
 * GB/s (16 n_floats bytes per pass over the mean pass time). Allocates and
 * frees 16 n_floats bytes of device memory on the current device; blocks
 * until done. n_floats in [1024, 2^34], reps >= 1, else WF_E_ARG. */
wf_status wf_stream_bandwidth(int64_t n_floats, int reps, double* gbs_out);

/* ------------------------------------------------------------------------ */
/* Serving engine: continuous batching of forward and gradient requests.     */
/* ------------------------------------------------------------------------ */

#define WF_REQ_FORWARD  0
#define WF_REQ_GRADIENT 1

typedef struct {
    int            kind;         /* WF_REQ_FORWARD or WF_REQ_GRADIENT            */
    wf_geom        geom;
    const float*   m_dev;        /* squared slowness, computational grid (device) */
    double         dt;
    int            nt;
    int            nsrc;
    const double*  src_xyz;      /* host, copied at submit                        */
    const float*   src_wav;      /* device [nt][nsrc]                             */
    int            nrec;
    const double*  rec_xyz;      /* host, copied at submit                        */
    const float*   d_obs;        /* device [nt][nrec], gradient requests only     */
    float*         rec_out;      /* device [nt][nrec]: modelled data (written)    */
    float*         grad_out;     /* device Nc^D, gradient requests only (written) */
    double*        misfit_out;   /* host, gradient requests only (written at completion) */
} wf_request;

/* Create an engine that may hold at most `hbm_budget_bytes` of device memory
 * for admitted requests and run at most `max_slots` requests at once. It owns
 * its own HIP streams on the current device and allocates the budget once, at
 * creation. A gradient request stores every forward wavefield when they fit in
 * a quarter of the budget, else keeps revolve checkpoints in that quarter
 * (results are the same bits either way). */
wf_status wf_engine_create(int64_t hbm_budget_bytes, int max_slots, wf_engine** out);

/* Queue a request; returns at once with a ticket. The request's device inputs
 * must be complete when the call is made (no work still writing them) and
 * stay valid and unchanged until the ticket is reported done. Requests that
 * could never fit the budget fail here with WF_E_BUDGET. The same as
 * wf_engine_submit_on(engine, req, NULL, 0, ticket). */
wf_status wf_engine_submit(wf_engine* engine, const wf_request* req, uint64_t* ticket);

/* Queue a request whose device inputs are produced by work on the caller's
 * `stream` (hipStream_t as void*, NULL the default stream): with ordered != 0
 * the call records an event on `stream` and every piece of the engine's work
 * on the request waits for it on the device, so the caller needs no
 * synchronisation between producing the inputs and submitting (work queued
 * on `stream` after the call is not waited for). Returns at once, as
 * wf_engine_submit, which it equals for ordered == 0. The inputs must stay
 * valid and unchanged until the ticket is reported done; outputs are complete
 * when it is. */
wf_status wf_engine_submit_on(wf_engine* engine, const wf_request* req, void* stream, int ordered,
                              uint64_t* ticket);

/* Device bytes the engine reserves from a budget of `hbm_budget_bytes` for
 * `req` when it admits it (its fields, coefficients, sparse and injection
 * tables, records and, for a gradient, the checkpoint memory it is given):
 * an upper bound on what serving the request allocates from the budget. A
 * request whose reservation exceeds the engine's budget is refused at
 * submission. Pure host function (reads the host coordinates). */
wf_status wf_engine_request_bytes(const wf_request* req, int64_t hbm_budget_bytes, int64_t* bytes);

/* Advance the engine: admit queued requests as slots and memory free up, issue
 * their next batch of steps, and report finished tickets (up to `cap`) with
 * their status. Non-blocking unless `wait_ms` > 0, in which case it waits up to
 * that long for at least one completion. */
wf_status wf_engine_poll(wf_engine* engine, uint64_t* done_tickets, wf_status* done_status,
                         int cap, int* n_done, int wait_ms);

/* Engine statistics: queued, running, completed counts and device bytes in use. */
wf_status wf_engine_stats(const wf_engine* engine, int64_t* queued, int64_t* running,
                          int64_t* completed, int64_t* bytes_in_use);

/* Completed requests by the path that ran them (any pointer may be NULL):
 * forward shots whose two wavefields fit one work-group's LDS (z padded to
 * 4, at most 40 640 floats for both: e.g. 141 x 141 in 2D, 26^3 in 3D) run
 * as resident teams, a work-group stepping a whole request in LDS with only
 * work-group barriers, or, when a launch holds few requests, each split
 * over up to 8 work-groups that recompute their neighbours' nearest planes
 * and exchange boundary planes every few updates (requests of one dimension
 * and order that are set up together share a launch; up to 4 launches run
 * at once);
 * other forward shots of at most 5 M nodes share batched step launches; the
 * rest, and every gradient, run on worker streams. Resident teams are on by
 * default; WAVEFD_TEAMS=0 in the environment at engine creation sends their
 * requests to the batched launches instead. Results are the same bits on
 * every path. WF_E_ARG if engine is NULL. */
wf_status wf_engine_paths(const wf_engine* engine, int64_t* teams, int64_t* batched, int64_t* workers);

/* Wait for every request, then free the engine. */
wf_status wf_engine_destroy(wf_engine* engine);

#ifdef __cplusplus
}
#endif

#endif /* WAVEFD_H */
