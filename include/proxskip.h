/*
 * proxskip.h -- C ABI of the MI355X (gfx950) library for TV-regularised parallel-beam tomography
 * solved by ProxSkip with the SVRG gradient estimator (ProxSVRGSkip).
 *
 * Problem (Sec. 2.1, Eq. 5, an instance of Eq. 1):
 *     min_x  1/2 ||A x - b||^2 + alpha TV(x) + I_{x >= 0}(x)
 * with A the discrete Radon transform, split into N subsets of interleaved angles
 * (A_i, b_i), i = 0..N-1, subset i holding the angles {i, i+N, i+2N, ...} (Sec. 1.2, the
 * data-splitting figure of Sec. 1.3).
 *
 * Conventions shared by every call:
 *   - Image x: [nz][ny][nx] row-major.  Pixel (i, j) has centre (j - (nx-1)/2, i - (ny-1)/2) in
 *     pixel units.  Slices are independent for the projector (parallel beam, rotation axis z).
 *   - Angles theta_k = k*pi/A (k = 0..A-1) unless a table is given.  Detector bin u has centre
 *     s_u = (u - (B-1)/2) * bin_width + det_offset; ray (k, u) is {x cos + y sin = s_u}.
 *   - Sinogram b: [nz][A][B].  A subset sinogram y_i: [nz][a_i][B], its angles in increasing
 *     order, a_i = number of k < A with k mod N == i.
 *   - Dual field (TV prox warm start): [d][nz][ny][nx], d = 2 when nz == 1 and d = 3 otherwise
 *     (3D TV couples slices).
 *   - Every floating-point buffer has the geometry's dtype (float or double).
 *   - Device pointers are HIP device memory owned by the caller, contiguous, aligned to at least
 *     the dtype size.  No compute call allocates or frees device memory: work buffers are
 *     passed in as a caller-owned workspace whose size the *_workspace_bytes queries return
 *     (device_alloc below is an optional allocator for them; the caller still owns the memory).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that launch kernels return
 *     as soon as the work is queued (stream-ordered); asynchronous faults surface at the next
 *     synchronisation.
 *   - Every call returns a ps_status; on failure last_error_message() (per thread) describes it.
 *     Argument checks run on the host before anything is queued.
 */
#ifndef PROXSKIP_H
#define PROXSKIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define PS_API __attribute__((visibility("default")))
#else
#define PS_API
#endif

typedef enum {
    PS_OK = 0,
    PS_EINVAL = -1,       /* invalid argument or workspace too small                         */
    PS_ENOMEM = -2,       /* host allocation failed                                           */
    PS_EHIP = -3,         /* a HIP runtime call or kernel launch failed                       */
    PS_EBUDGET = -4,      /* reserved for admission control above this library                */
    PS_ENONFINITE = -5,   /* a non-finite iterate was detected at an epoch end                */
    PS_ECANCELLED = -6,   /* the solver handle was cancelled                                  */
    PS_EUNSUPPORTED = -7  /* shape outside what the kernels support (a side > 4096, B > 2048) */
} ps_status;

typedef enum { PS_F32 = 0, PS_F64 = 1 } ps_dtype;

/* Parallel-beam geometry (Sec. 2.1: discrete Radon transform; Sec. 1.2: angle subsets). */
typedef struct {
    int32_t nx, ny, nz;      /* image columns, rows, slices (nz = 1 for 2D)                    */
    int32_t n_angles;        /* A >= 1                                                          */
    const double *angles;    /* optional host table of A angles in radians (copied); NULL =>   */
                             /* uniform k*pi/A                                                  */
    int32_t n_bins;          /* B >= 1                                                          */
    double bin_width;        /* detector bin width in pixel units, > 0 (1.0 = pixel width)      */
    double det_offset;       /* detector centre offset in pixel units                           */
    int32_t n_subsets;       /* N >= 1, at most A                                               */
    ps_dtype dtype;          /* precision of every buffer and of the arithmetic                 */
} ps_geometry_desc;

typedef struct ps_geometry ps_geometry;  /* opaque; immutable after geometry_upload            */

/* Validate `desc` and build the host-side geometry (per-angle tables, launch plans).
 * No device work.  Errors: PS_EINVAL (bad sizes, N > A, bin_width <= 0), PS_EUNSUPPORTED. */
PS_API ps_status make_geometry(const ps_geometry_desc *desc, ps_geometry **out);
PS_API void free_geometry(ps_geometry *geom);

/* Bytes of device memory the geometry's per-angle tables need. */
PS_API size_t geometry_device_bytes(const ps_geometry *geom);

/* Copy the per-angle tables into caller-owned device memory `dev_buf` (at least
 * geometry_device_bytes bytes, 256-byte aligned), stream-ordered.  The geometry keeps the
 * pointer: `dev_buf` must outlive every call made with this geometry. */
PS_API ps_status geometry_upload(ps_geometry *geom, void *dev_buf, size_t bytes, void *stream);

/* a_i, the number of angles in subset i; subset = -1 => A.  Returns -1 for a bad subset. */
PS_API int32_t subset_size(const ps_geometry *geom, int32_t subset);

/* Launch plan of a geometry: tile shapes and work splits of the kernels.  A field of 0 means
 * "chosen by the library from the shape".  A plan changes how work is divided, never what is
 * computed: results differ only by the order of floating-point sums (a different ray split or
 * angle grouping), within the documented tolerances.  Workspace sizes depend on the plan: set it
 * (or autotune) before sizing workspaces and creating solver handles.
 *   proj_split_*   workgroups along each ray (projector; partial sums added by a second pass)
 *   bp_groups_*    angle groups of the backprojector (each writes its own partial image)
 *   bp_strip_*     image rows (or columns) per backprojector workgroup: 8, 4, 2 or 1
 *   fgp_iters      inner iterations per 2D FGP launch (temporal blocking): 1..16 (FP32) or
 *                  1..8 (FP64), 0 = 8; capped at (fgp_waves x fgp_rows) / 2 - 2 so that every
 *                  tile keeps interior rows
 *   bp_method_*    1 = ray-driven scatter into LDS strips + combine pass; 2 = pixel-driven gather
 *                  with the update fused (needs bins at least one pixel apart along every ray's
 *                  stepping axis, e.g. bin_width >= 1; otherwise scatter is used)
 *   bp_gather_rows rows per wave of the gather's tiles (63 columns x 4 waves x rows): 2 or 4
 *   bp_gather_split waves of a gather workgroup that share one block of rows, each taking every
 *                  split-th angle (their sums added in LDS in wave order): 1, 2 or 4; the tile
 *                  is then 63 columns x (4 / split) x rows.  0 = automatic: 4 when the
 *                  unsplit tiles number fewer than 256, 2 below 1024, else 1.
 *   fgp_cols       2D FGP columns per lane: 1 (tiles 64 columns wide) or 2 (128 wide: the halo
 *                  of T + 1 columns per side is a smaller share); 0 = automatic (1).  Does not
 *                  change results, not even their rounding.
 *   bp_gather_fused inside solver iterations that backproject subsets with the gather while the
 *                  projector splits rays: 2 = the gather adds the projector's partial sums itself
 *                  as it stages the ray values (no reduction pass: one launch fewer per
 *                  iteration), 1 = the reduction pass runs; 0 = automatic (2 for splits up to
 *                  8 whose partials take at most 32 MiB).  Same results either way, to the bit.
 *                  get_plan reports 2 only where it takes effect.
 *   fgp3d_chunk    slices each workgroup of the 3D FGP marches through: 1..256, 0 = automatic
 *                  (4 for one iteration per launch, 16 for two)
 *   fgp_waves, fgp_rows  2D FGP tile: waves per workgroup and image rows per wave, one of
 *                  (4,4) (4,8) (8,2) (8,4) (8,8) (16,2) (16,4); both 0 = automatic (8,4 FP32;
 *                  16,2 FP64).  The tile does not change results, not even their rounding.
 *                  fgp_iters and the tile apply to a prox computed alone: the proxes of several
 *                  handles advanced together (solver_epochs / solver_steps over several
 *                  handles) share launches on the automatic tile and depth.
 *   fgp3d_form     3D FGP launches: 1 = one inner iteration per launch (62 x 14 tiles); 2..5 =
 *                  two per launch (7 values read and 6 written per voxel for two iterations
 *                  instead of 20) on tiles of 8 waves x 2 rows (2), 4 x 4 (3), both 60 x 12
 *                  outputs, 16 x 2 (4) or 8 x 4 (5), both 60 x 28 outputs; 0 = automatic (5 FP32,
 *                  2 FP64).  The form does not change results, not even their rounding.
 * "_full" applies to all-angle calls (subset = -1), "_subset" to single subsets. */
typedef struct {
    int32_t proj_split_full, proj_split_subset;
    int32_t bp_groups_full, bp_groups_subset;
    int32_t bp_strip_full, bp_strip_subset;
    int32_t fgp_iters;
    int32_t bp_method_full, bp_method_subset;
    int32_t bp_gather_rows;
    int32_t fgp3d_chunk;
    int32_t fgp_waves, fgp_rows;
    int32_t fgp3d_form;
    int32_t bp_gather_split;
    int32_t fgp_cols;
    int32_t bp_gather_fused;
} ps_plan;

/* The plan in effect (automatic choices filled in) / replace the overrides.  set: fields out of
 * range => PS_EINVAL and nothing changes. */
PS_API ps_status geometry_get_plan(const ps_geometry *geom, ps_plan *out);
PS_API ps_status geometry_set_plan(ps_geometry *geom, const ps_plan *plan);

/* Autotuner: time candidate plans of the projector, backprojector and 2D FGP on this geometry
 * (HIP events on `stream`; per candidate one warm-up launch, then the median of three rounds of
 * `reps` launches; synthetic inputs), keep the fastest of each -- a candidate must beat the
 * automatic plan by 3% to replace it -- store them as the geometry's plan and return it in
 * `out`.
 * Synchronises `stream`.  workspace: device scratch of geometry_autotune_workspace_bytes bytes.
 * The geometry must be uploaded.  Errors: PS_EINVAL, PS_EHIP. */
PS_API size_t geometry_autotune_workspace_bytes(const ps_geometry *geom);
PS_API ps_status geometry_autotune(ps_geometry *geom, void *workspace, size_t ws_bytes,
                            int32_t reps, void *stream, ps_plan *out);

/* Forward projection y = A_i x (Sec. 1.2: the subset operator A_i), ray-driven Joseph
 * interpolation.  subset = -1 projects all A angles (y = [nz][A][B]).
 * x: device [nz][ny][nx]; y: device [nz][a_i][B], overwritten.
 * workspace: device scratch of at least project_workspace_bytes(geom, subset) bytes (may be
 * NULL when that is 0).  Errors: PS_EINVAL, PS_EHIP. */
PS_API size_t project_workspace_bytes(const ps_geometry *geom, int32_t subset);
PS_API ps_status project_subset(const ps_geometry *geom, int32_t subset, const void *x, void *y,
                         void *workspace, size_t ws_bytes, void *stream);

/* Backprojection x = A_i^T y (accumulate = 0) or x += A_i^T y (accumulate = 1): the exact
 * adjoint of project_subset -- every ray deposits its value times the projector's own two
 * interpolation weights along the same walk (results reproducible bit for bit).
 * y: device [nz][a_i][B]; x: device [nz][ny][nx].  workspace: device scratch of at least
 * backproject_workspace_bytes(geom, subset) bytes (partial images).
 * Errors: PS_EINVAL (bad subset, pointers, workspace too small), PS_EHIP. */
PS_API size_t backproject_workspace_bytes(const ps_geometry *geom, int32_t subset);
PS_API ps_status backproject_subset(const ps_geometry *geom, int32_t subset, const void *y, void *x,
                             int32_t accumulate, void *workspace, size_t ws_bytes, void *stream);

/* Proximal operator of g = TV + I_C (Eq. 3 with the regulariser of Eq. 5), with weight tau:
 *     z = argmin_z 1/2 ||z - v||^2 + tau TV(z) + I_C(z),   C = {z >= 0} if nonneg else R^n,
 * isotropic TV with forward differences (zero last difference), solved by n_inner iterations of
 * FGP (Beck & Teboulle 2009), warm-started from `dual` (Sec. 2.1: a fixed number of
 * warm-started inner iterations).
 * v, z: device [nz][ny][nx]; z may alias v.  dual: device [d][nz][ny][nx], in = warm start,
 * out = final dual; NULL => cold start from zeros and not returned.  tau == 0 => z = P_C(v),
 * dual untouched.  workspace: at least tv_prox_workspace_bytes(geom) bytes.
 * Errors: PS_EINVAL (tau < 0, n_inner < 0, workspace too small), PS_EHIP. */
PS_API size_t tv_prox_workspace_bytes(const ps_geometry *geom);
PS_API ps_status tv_prox_fgp(const ps_geometry *geom, const void *v, void *z, double tau,
                      int32_t n_inner, int32_t nonneg, void *dual, void *workspace,
                      size_t ws_bytes, void *stream);

/* Gradient estimators G_k of the table beside Algorithm 1 (Sec. 1.2). */
typedef enum {
    PS_EST_SVRG = 0,   /* N (grad f_i(x) - grad f_i(xs)) + grad f(xs), xs refreshed every N iterations */
    PS_EST_LSVRG = 1,  /* the same G, xs refreshed with probability 1/N per iteration (loopless)     */
    PS_EST_SAGA = 2    /* N (grad f_i(x) - v_i) + sum_j v_j with the table v of Eq. 4              */
} ps_estimator;

/* Parameters of Algorithm 1 (Sec. 1.2). */
typedef struct {
    double gamma;             /* step size > 0 (the paper uses 1/L, L = ||A||^2)                */
    double p;                 /* prox probability, 0 < p <= 1                                   */
    double alpha;             /* TV weight >= 0                                                  */
    int32_t fgp_inner;        /* FGP iterations per prox call >= 0                              */
    int32_t nonneg;           /* 1 => g includes I_{x >= 0}                                      */
    int32_t n_epochs;         /* epochs to run (1 epoch = N iterations = one data pass)         */
    int32_t plain_prox_svrg;  /* 1 => non-skipped ProxSVRG: x+ = prox_{gamma g}(x - gamma G),   */
                              /*      h untouched                                                */
    uint64_t seed;            /* seed of the subset and coin streams                            */
    int64_t k0;               /* first iteration index (resume point), a multiple of N          */
    double tol_rel_change;    /* > 0 => stop at the first epoch end with                        */
                              /*   ||x_e - x_{e-1}|| / ||x_e|| < tol; 0 => run n_epochs         */
    int32_t estimator;        /* ps_estimator (0 = SVRG)                                        */
} ps_solver_params;

typedef struct {
    int32_t epochs_done;      /* epochs completed by the last run / since solver_init           */
    int32_t iters_done;       /* iterations completed (k - k0)                                  */
    int32_t prox_calls;       /* prox evaluations (coin flips theta_k = 1)                      */
    double last_rel_change;   /* ||x_e - x_{e-1}|| / ||x_e|| at the last completed epoch end   */
} ps_solver_stats;

/* ProxSkip (Algorithm 1) with the estimator params->estimator:
 *   PS_EST_SVRG (ProxSVRGSkip row of its table): every N iterations (k mod N == 0) snapshot
 *     xs = x_k, gs = grad f(xs) = A^T (A xs - b);  G_k = N (grad f_i(x_k) - grad f_i(xs)) + gs
 *   PS_EST_LSVRG (ProxLSVRGSkip): the same G_k; the snapshot is refreshed at the run's first
 *     iteration and at every later k with rho_k = 1 (sample_refresh_coins), before G_k is formed
 *   PS_EST_SAGA (ProxSAGASkip, Eq. 4): G_k = N (grad f_i(x_k) - v_i) + vbar, then
 *     vbar += grad f_i(x_k) - v_i and v_i = grad f_i(x_k); the table is filled with
 *     v_j = grad f_j(x_k0) and vbar = sum_j v_j (increasing j) at the run's first iteration
 * then, with i = i_k uniform on {0..N-1},
 *   xh   = x_k - gamma (G_k - h_k)
 *   theta_k ~ Bernoulli(p): x_{k+1} = prox_{(gamma/p) g}(xh - (gamma/p) h_k) if theta_k = 1,
 *                           else x_{k+1} = xh
 *   h_{k+1} = h_k + (p/gamma)(x_{k+1} - xh)
 * with g = alpha TV + I_C, the prox by tv_prox_fgp with fgp_inner warm-started iterations, and
 * i_k, theta_k from sample_sequences(seed, ...).
 * b: device [nz][A][B].  x, h, dual: device, in = state at k0 (zeros for a fresh run),
 * out = state after the run.  For SVRG, (x, h, dual, k) is the complete resumable state; the
 * loopless-SVRG snapshot and the SAGA table live in the workspace, so a new run from k0 > 0
 * starts them afresh at x_k0 (a handle keeps them across solver_epochs calls).
 * workspace: at least proxskip_workspace_bytes(geom, params) bytes.  stats_out may be NULL.
 * Synchronises `stream` once at the end (and at every epoch end when tol_rel_change > 0).
 * Errors: PS_EINVAL, PS_EHIP, PS_ENONFINITE. */
PS_API size_t proxskip_workspace_bytes(const ps_geometry *geom, const ps_solver_params *params);
PS_API ps_status proxskip_svrg_run(const ps_geometry *geom, const void *b, void *x, void *h,
                            void *dual, const ps_solver_params *params,
                            ps_solver_stats *stats_out, void *workspace, size_t ws_bytes,
                            void *stream);

/* proxskip_svrg_run for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same iteration and
 * arguments, and bit for bit the same results, without a workspace.  The solver's scratch lives
 * in a fixed device array of the library, proxskip_noalloc_max_bytes() bytes (64 MiB), one per
 * GPU, held from the first call on that GPU until the process ends; its device address is taken
 * once per device on the first call there (the caller's current device is used).  The call makes
 * no device allocation.
 * Limits: proxskip_workspace_bytes(geom, params) must not exceed proxskip_noalloc_max_bytes()
 * (a 512^2 FP32 solve with 720 x 768 data fits), else PS_EINVAL; tol_rel_change must be 0 (a
 * fixed number of epochs), else PS_EINVAL.
 * Every call on one GPU uses the same array, which keeps the last call's contents (nothing in it
 * has to start at zero): calls that overlap on one GPU (other streams, other host threads) race
 * and must be serialised by the caller.  Synchronises `stream` once at the end.
 * Errors: PS_EINVAL, PS_EHIP, PS_ENONFINITE. */
PS_API size_t proxskip_noalloc_max_bytes(void);
PS_API ps_status proxskip_svrg_run_noalloc(const ps_geometry *geom, const void *b, void *x, void *h,
                                    void *dual, const ps_solver_params *params,
                                    ps_solver_stats *stats_out, void *stream);

/* Resumable solver handles (the same iteration as proxskip_svrg_run, split into calls), and
 * batching of independent problems.
 * solver_init binds caller-owned buffers (they must outlive the handle; the workspace must be
 * proxskip_workspace_bytes(geom, params) bytes and may not be shared between live handles).
 * solver_epochs runs up to n_epochs further epochs of every handle on `stream`.  The handles may
 * have different geometries, sizes, subset counts, dtypes and parameters: they advance in
 * lockstep, one iteration each per step, and every stage of a step (snapshot copies,
 * projections, backprojections with the fused update, FGP launches, epoch-end norms) is one
 * launch over a work list of up to 16 handles.  Each handle computes exactly what it computes
 * alone (bit for bit).  A handle with tol_rel_change > 0 pauses at each epoch end until its
 * norms reach the host (pinned host memory behind an event) while the others continue; handles
 * that met their tolerance or epoch budget are skipped.  Returns once every handle is done with
 * this call's epochs (synchronising only for tolerance checks).  A handle may appear once.
 * solver_query synchronises the handle's stream and reports its progress.
 * solver_cancel makes later solver_epochs calls on the handle return PS_ECANCELLED. */
typedef struct ps_solver ps_solver;
PS_API ps_status solver_init(const ps_geometry *geom, const void *b, void *x, void *h, void *dual,
                      const ps_solver_params *params, void *workspace, size_t ws_bytes,
                      ps_solver **out);
PS_API ps_status solver_epochs(ps_solver *const *handles, int32_t n_handles, int32_t n_epochs,
                        void *stream);
/* solver_steps: the same lockstep, bounded by steps instead of epochs: every handle that can
 * still advance (epoch budget not spent, tolerance not met, not cancelled) does at most n_steps
 * iterations, crossing epoch ends as it goes.  A serving loop calls it in rounds and admits new
 * handles between rounds.  Returns with every tolerance check settled. */
PS_API ps_status solver_steps(ps_solver *const *handles, int32_t n_handles, int32_t n_steps,
                       void *stream);
/* solver_epochs_graph: the same epochs as solver_epochs, issued as HIP graphs.  Each round (one
 * epoch of every handle that still runs; handles with fewer subsets wait for the round's end) is
 * captured on a library-owned stream, instantiated -- or, when an earlier round had the same
 * launch topology (handles, subset counts, coin pattern), that executable graph is updated with
 * the new kernel arguments -- and launched on `stream`.  The graphs are cached in handles[0]
 * (at most 64, released by solver_free).  Every handle must be at an epoch start (k a multiple
 * of N), else PS_EINVAL.  Results are bit for bit those of solver_epochs. */
PS_API ps_status solver_epochs_graph(ps_solver *const *handles, int32_t n_handles, int32_t n_epochs,
                              void *stream);
/* 1 when the handle will not advance any further (converged, budget spent, cancelled or
 * non-finite) and nothing of it is pending on the host side, 0 otherwise, -1 for NULL.  Does not
 * synchronise. */
PS_API int32_t solver_done(const ps_solver *handle);
PS_API ps_status solver_query(ps_solver *handle, ps_solver_stats *stats_out);
PS_API ps_status solver_cancel(ps_solver *handle);
PS_API void solver_free(ps_solver *handle);

/* Host-side random streams (the library's own counter-based SplitMix64):
 *   u(seed, j) = mix64(seed + (j + 1) * 0x9e3779b97f4a7c15)   (Steele, Lea & Flood 2014)
 *   i_k = ((u(seed, 2k) >> 32) * N) >> 32,  theta_k = (u(seed, 2k+1) >> 11) < floor(p * 2^53)
 * for k = k0 .. k0+count-1 (Sec. 1.2 "sampling i_k"; Algorithm 1: theta_k ~ Bernoulli(p)).
 * Either output may be NULL.  Errors: PS_EINVAL. */
PS_API ps_status sample_sequences(uint64_t seed, int64_t k0, int64_t count, int32_t n_subsets,
                           double p, int32_t *subset_out, uint8_t *coin_out);

/* Refresh coins of the loopless SVRG estimator (Sec. 1.2: the full gradient is refreshed with
 * probability 1/N in every iteration), from the same generator at counters 2^62 + k:
 *   rho_k = (u(seed, 2^62 + k) >> 11) < floor(2^53 / N),   k = k0 .. k0+count-1.
 * Errors: PS_EINVAL. */
PS_API ps_status sample_refresh_coins(uint64_t seed, int64_t k0, int64_t count, int32_t n_subsets,
                               uint8_t *out);

/* FISTA (Beck & Teboulle 2009; the table beside Algorithm 1: ISTA with an acceleration step),
 * with the full gradient and the same prox as Algorithm 1:
 *   x_{k+1} = prox_{gamma g}(y_k - gamma A^T (A y_k - b)),  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
 *   y_{k+1} = x_{k+1} + ((t_k - 1) / t_{k+1}) (x_{k+1} - x_k),   y_0 = x_0,  t_0 = 1.
 * b: device [nz][A][B].  x: device, in x_k, out x_{k+n_iters}.  y: device [nz][ny][nx], in y_k,
 * out y_{k+n_iters} (a copy of x_0 for a fresh run).  t: host, in t_k, out t_{k+n_iters} (1 for
 * a fresh run).  dual: device [d][nz][ny][nx] FGP warm start, in/out (zeros for a fresh run).
 * (x, y, dual, t) is the complete state: consecutive calls continue one run.
 * workspace: at least fista_workspace_bytes(geom) bytes.  Stream-ordered; does not
 * synchronise.  Errors: PS_EINVAL, PS_EHIP. */
PS_API size_t fista_workspace_bytes(const ps_geometry *geom);
PS_API ps_status fista_run(const ps_geometry *geom, const void *b, void *x, void *y, void *dual,
                    double *t, double gamma, double alpha, int32_t fgp_inner, int32_t nonneg,
                    int32_t n_iters, void *workspace, size_t ws_bytes, void *stream);

/* High-accuracy reference solution x* of Eq. 5 (Sec. 2.1: computed with a separate primal-dual
 * method, PDHG with diagonal preconditioning, Chambolle & Pock 2011, as in the data-splitting
 * figure), with K = [A; D]:
 *   tau = 1 / (column sums of |K|),  sigma = 1 / (row sums of A) (1 on empty rays), 1/2 on D
 *   x+   = P_C(x - tau (A^T y1 + D^T y2)),   xbar = 2 x+ - x
 *   y1+  = (y1 + sigma (A xbar - b)) / (1 + sigma)
 *   y2+  = y2 + D xbar / 2, each pixel's d-vector scaled onto the ball of radius alpha
 * b: device [nz][A][B].  x [nz][ny][nx], y1 [nz][A][B], y2 [d][nz][ny][nx]: device, in/out (zeros
 * for a fresh start; (x, y1, y2) is the complete state, so runs may be continued).
 * workspace: at least pdhg_workspace_bytes(geom) bytes.  Stream-ordered; does not synchronise.
 * Errors: PS_EINVAL, PS_EHIP. */
PS_API size_t pdhg_workspace_bytes(const ps_geometry *geom);
PS_API ps_status pdhg_run(const ps_geometry *geom, const void *b, void *x, void *y1, void *y2,
                   double alpha, int32_t nonneg, int32_t n_iters, void *workspace,
                   size_t ws_bytes, void *stream);

/* Optional allocator for large caller-owned buffers such as workspaces (not part of the method).
 * Many-GiB allocations made after many earlier allocations and frees can consist of small
 * physical pieces; kernels that stream several such arrays at once (the 3D FGP iteration walks
 * thirteen) then stall on address translation.  device_alloc(bytes, device, &ptr, &contiguous)
 * requests physically contiguous device memory on `device` and falls back to an ordinary
 * allocation when the driver cannot provide it; *contiguous (may be NULL) tells which.  The
 * memory is uninitialised and owned by the caller, who releases it with device_free, which first
 * waits for all work on that device (a buffer may still be in use by queued kernels).
 * device_free(NULL) does nothing.  The current device is unchanged on return.
 * Errors: PS_EINVAL (bytes == 0, out == NULL, no such device, not device memory), PS_EHIP
 * (the ordinary allocation failed too). */
PS_API ps_status device_alloc(size_t bytes, int32_t device, void **out, int32_t *contiguous);
PS_API ps_status device_free(void *ptr);

/* Measurement support (not part of the method): the GPU time of chosen classes of kernel launches
 * inside later calls on any stream, from HIP events recorded on the launching stream right before
 * and after each launch of a chosen class (the interval covers the kernel's execution and its
 * dispatch).  A launch over a work list counts in the class of its first item.  Launches into a
 * stream being captured as a graph are not timed; at most 16384 launches per class are.
 * kernel_timer_start(mask): forget earlier timings and time the classes whose bit (1 << class)
 * is set.  kernel_timer_read: synchronises the class's events and returns their summed time and
 * count.  kernel_timer_stop: stop timing (what was timed can still be read).
 * Errors: PS_EINVAL (unknown class), PS_EHIP. */
typedef enum {
    PS_KC_BACKPROJECT_SUBSET = 1,  /* scatter backprojector, subset launches                     */
    PS_KC_BACKPROJECT_FULL = 2,    /* scatter backprojector, all-angle launches                  */
    PS_KC_PROJECT_SUBSET = 3,      /* projector, subset launches                                 */
    PS_KC_PROJECT_FULL = 4,        /* projector, all-angle launches                              */
    PS_KC_BACKPROJECT_COMBINE = 5, /* the scatter's combine pass (partial images + epilogue)     */
    PS_KC_PROJECT_REDUCE = 6,      /* the projector's split-ray sum                              */
    PS_KC_BACKPROJECT_GATHER = 7,  /* pixel-driven backprojector                                 */
    PS_KC_FGP2D = 8,               /* 2D FGP launches                                            */
    PS_KC_FGP3D = 9                /* 3D FGP iteration launches                                  */
} ps_kernel_class;
PS_API ps_status kernel_timer_start(uint32_t class_mask);
PS_API ps_status kernel_timer_read(int32_t kernel_class, double *total_ms, int32_t *launches);
PS_API ps_status kernel_timer_stop(void);

/* Measurement support: the average GPU time of one launch of one kernel class alone, with the
 * geometry's plan on synthetic inputs: HIP events on `stream` around `reps` back-to-back launches,
 * the median of three rounds (each launch's dispatch overlaps the previous launch, as inside a
 * solve).  Classes: PS_KC_BACKPROJECT_SUBSET / _FULL (the scatter kernel without its combine
 * pass; the plan must take the scatter for that call), PS_KC_BACKPROJECT_GATHER (subset 0; the
 * plan must take the gather), PS_KC_PROJECT_SUBSET / _FULL (the projector kernel without the
 * split-ray sum; subset launches read the two images x and xs, or one image where the solver
 * keeps their difference, as the solver's do).  Subset launches use subset 0.  workspace: kernel_time_workspace_bytes(geom)
 * bytes.  Synchronises `stream`.  Errors: PS_EINVAL, PS_EHIP. */
PS_API size_t kernel_time_workspace_bytes(const ps_geometry *geom);
PS_API ps_status kernel_time(const ps_geometry *geom, int32_t kernel_class, int32_t reps,
                      void *workspace, size_t ws_bytes, void *stream, double *us_per_launch);

/* Description of the last error on the calling thread ("" if none). */
PS_API const char *last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* PROXSKIP_H */
