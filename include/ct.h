/*
 * ct.h -- C ABI of the MI355X block-iterative CT solver (CSGD / GCSGD).
 *
 * The library solves the linear inverse problem y = A x + e (Eq. 1/2) by the
 * randomised block scheme of Alg. 4-6: every update picks a column block J
 * (a voxel cuboid) and a group of row blocks I_G (detector tiles of some
 * views), back-projects g_J = (A_{I_G}^J)^T r_{I_G} (Eq. 7), takes the
 * relaxed exact line-search step mu = beta ||g||^2 / ||A g||^2 (Eq. 11 with
 * the relaxation of Sec. II-B) and records the partial projection
 * z^J_{I_G} = A_{I_G}^J (x_J + mu g_J); the residual is rebuilt as
 * r = y - sum_j z^j on the touched rows (Sec. II-C), and every updated block
 * is set to the mean of its updates at the end of an epoch.
 * A_ij, the intersection length of ray i with voxel j (Sec. II-A), is never
 * stored: every projection recomputes it on the fly.
 *
 * Conventions
 *  - Every function returns CT_OK (0), an error (< 0) or information (> 0).
 *    ct_last_error() gives a thread-local message for the last failure.
 *    Argument errors are detected before any device work is enqueued, so a
 *    rejected call writes nothing.
 *  - Device work is asynchronous on the caller's HIP stream, passed as
 *    `void* stream` (NULL = the default stream).  Device pointers passed in
 *    (x, y, r, g, workspace) stay owned by the caller; they must remain valid
 *    until the stream reaches the enqueued work.  Execution errors surface at
 *    the next synchronising call.
 *  - Handles (ct_geom, ct_schedule, ct_solver, ct_batch) are owned by the
 *    library and released by the matching destroy call.  Geometry and
 *    schedule handles hold small read-only device tables that the library
 *    allocates on the current device; the large per-job state (z, r, g ...)
 *    lives in caller-allocated workspace.
 *  - Units: lengths in mm, x in mm^-1.  Layouts (row-major, last index
 *    fastest): x[nz][ny][nx]; y, r[n_views][nv][nu]; z[n_col][n_views][nv][nu].
 *  - All device arrays are float32; the step size and the norms it needs are
 *    reduced in float64.
 */
#ifndef CT_H
#define CT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CT_OK 0
#define CT_NOT_CONVERGED 1     /* ct_solve hit its epoch cap              */
#define CT_EINVAL (-1)         /* bad argument; nothing was enqueued      */
#define CT_ENOMEM (-2)         /* device allocation failed                */
#define CT_EDEVICE (-3)        /* HIP runtime error                       */
#define CT_EUNSUPPORTED (-4)   /* valid but not implemented combination   */

/* ---- geometry ------------------------------------------------------------
 * Scan geometries (Sec. II-D: arbitrary source/detector poses per view theta,
 * detector perpendicular to the source-to-detector-centre line).
 * views[k*12 + 0..11] = a | c | e_u | e_v (float64):
 *   CT_PAR2D        a = ray direction; ray of bin iu passes c + u e_u.
 *   CT_FAN2D_FLAT   a = source; ray from a through c + u e_u.
 *   CT_FAN2D_CURVED a = source; ray from a with direction
 *                   cos(u) n + sin(u) e_u, n = (c - a)/|c - a|, u in radians.
 *   CT_CONE3D_FLAT  a = source; ray from a through c + u e_u + v e_v.
 * with u = (iu - (nu-1)/2) pu and v = (iv - (nv-1)/2) pv.  2D kinds use
 * components 0 and 1 only and need nz = nv = 1.  e_u (and e_v) must be unit,
 * and for divergent kinds perpendicular to c - a (and to each other).
 * Ray index i = (view*nv + iv)*nu + iu; voxel index j = (iz*ny + iy)*nx + ix;
 * voxel (ix,iy,iz) is the half-open box [o + i h, o + (i+1) h).
 *
 * Row blocks (the sets I of Eq. 4) are lists of detector tiles
 * (view, u0, u1, v0, v1) (half-open index ranges); tiles of all row blocks must
 * partition the rays.  Column blocks (the sets J) are voxel boxes
 * (x0, x1, y0, y1, z0, z1) that must partition the volume.  The rays of a row
 * block are ordered tile by tile, v then u.
 */
enum { CT_PAR2D = 0, CT_FAN2D_FLAT = 1, CT_FAN2D_CURVED = 2, CT_CONE3D_FLAT = 3 };

typedef struct ct_geom_desc {
    int32_t kind;
    int32_t nx, ny, nz;
    double vx, vy, vz;          /* voxel pitch (mm)                      */
    double ox, oy, oz;          /* volume min corner (mm)                */
    int32_t n_views, nu, nv;
    double pu, pv;              /* bin pitch: mm, or rad for curved u    */
    const double* views;        /* host, n_views*12                      */
    int32_t n_row_blocks;
    const int32_t* rb_ptr;      /* host, n_row_blocks+1 tile offsets     */
    const int32_t* tiles;       /* host, rb_ptr[n_row_blocks]*5          */
    int32_t n_col_blocks;
    const int32_t* boxes;       /* host, n_col_blocks*6                  */
} ct_geom_desc;

typedef struct ct_geom ct_geom;

typedef struct ct_geom_info {
    int64_t n_rays, n_vox;
    int32_t m, n;               /* row and column block counts           */
    int32_t max_rb_rays;        /* largest row block (rays)              */
    int32_t max_cb_vox;         /* largest column block (voxels)         */
} ct_geom_info;

/* Validates the description and copies it (host arrays may be freed on
 * return).  The device tables (float64 per-view frames, per-ray 2D constants,
 * tile and ray-chunk lists) are built on the first call that needs them, on
 * the device current at that time; every later call on the geometry must run
 * with that device current.  CT_EINVAL on inconsistent sizes, non-partitions,
 * non-unit or non-perpendicular axes, or a volume not entirely in front of a
 * source.  Host-only. */
int ct_geom_create(const ct_geom_desc* desc, ct_geom** out);
void ct_geom_destroy(ct_geom* geom);
int ct_geom_get_info(const ct_geom* geom, ct_geom_info* out);

/* nnz(A_I^J) for every (row block, column block): the number of ray-voxel
 * pairs whose intersection length exceeds tau (mm) -- the block density that
 * drives the importance sampling of Sec. II-C (reading C6).  host_nnz is a
 * host array [m][n] (row-block major).  Synchronous on `stream`. */
int ct_geom_block_nnz(ct_geom* geom, double tau, int64_t* host_nnz, void* stream);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): ct_geom_block_nnz with its
 * counters in a static device array of the library (CT_NNZ_STATIC_MAX
 * entries of 8 bytes; each GPU the library runs on holds its own copy until
 * the process ends) instead of the geometry's tables, and the counts copied
 * straight into host_nnz.  It allocates nothing, on the device or the host:
 * the geometry's device tables must already be on the current device (any
 * earlier call that launches work on the geometry uploads them), else
 * CT_EINVAL.  CT_EINVAL when m * n > CT_NNZ_STATIC_MAX, before anything is
 * enqueued.  Every call on a GPU shares that GPU's array (cleared by a kernel
 * at the start of each call): calls that overlap on one GPU race.
 * Synchronous on `stream`. */
#define CT_NNZ_STATIC_MAX 65536
int ct_geom_block_nnz_static(ct_geom* geom, double tau, int64_t* host_nnz, void* stream);
/* The paper's own density estimate (Sec. II-C, Alg. 5): host_area[I*n + J] =
 * P_S, the area (detector units: mm, radians on a curved detector, mm^2 in
 * 3D) that the projection of column block J's box covers on the tiles of row
 * block I, summed over its views; computed exactly (hull of the projected
 * box corners, intersected with each tile's rectangle of bin edges) on the
 * host in float64.  Normalised per column (P = P_S / sum_I P_S) it feeds
 * ct_schedule_create_w.  host_area: caller memory of m*n doubles. */
int ct_geom_block_area(const ct_geom* geom, double* host_area);

/* ---- block projectors (Alg. 3) ---------------------------------------------
 * ct_block_fwd:  y_{I} (= or +=) A_I^J x_J   for I = union of row_blocks.
 *   Reads only x[J]; writes only the rays of the listed row blocks of y
 *   (full-size ray array [n_views][nv][nu]).
 * ct_block_back: g_J (= or +=) (A_I^J)^T r_I  (Eq. 7).
 *   Reads only the listed rays of r; writes only the voxels of J in g
 *   (full-size volume array).
 * row_blocks: host array of n_rb distinct row-block ids.  flags: CT_ACCUMULATE
 * adds instead of overwriting.  Lengths are computed in float32 from float64
 * ray frames; accumulation is float32. */
#define CT_ACCUMULATE 1
int ct_block_fwd(ct_geom* geom, const int32_t* row_blocks, int32_t n_rb, int32_t col_block,
                 const float* x, float* y, int32_t flags, void* stream);
int ct_block_back(ct_geom* geom, const int32_t* row_blocks, int32_t n_rb, int32_t col_block,
                  const float* r, float* g, int32_t flags, void* stream);

/* ---- schedule (Alg. 5 / Alg. 6 sampling) -----------------------------------
 * Drawn entirely up front: it depends on P(I,J), the parameters and the seed
 * only.  Per epoch: a uniform permutation of the column blocks, of which
 * ceil(gamma n) are used; for each, ceil(alpha m) successive draws without
 * replacement of row blocks with weight P(I,J) (zero weight never drawn),
 * cut into consecutive groups of group_size; beta_G = b sum_{I in G} P(I,J).
 * Uniform sampling gives every row block weight 1.  Mixed sampling
 * (Sec. III-D) gives row block I the weight P_I + theta (P_max - P_I), with
 * theta = min(1, epoch*theta_step) and P_max the largest P(., J) among the
 * row blocks of I's projection: row blocks whose tiles cover the same set of
 * views are the sub-detector areas of one projection.  A sub-area that J's
 * shadow misses gets theta P_max; a projection J does not reach keeps weight
 * 0.  beta always uses P.
 * Random numbers: SplitMix64 as a counter-based generator,
 * u64 = mix(seed + (ctr+1) * 0x9E3779B97F4A7C15), ctr = epoch*2^32 + k. */
enum { CT_SAMPLE_DENSITY = 0, CT_SAMPLE_UNIFORM = 1, CT_SAMPLE_MIXED = 2 };

typedef struct ct_sched_params {
    int32_t epochs;
    double alpha;               /* fraction of row blocks per column block */
    double gamma;               /* fraction of column blocks per epoch     */
    int32_t group_size;         /* s                                       */
    double b;                   /* beta = b * P_S/P_T                      */
    int32_t sampling;           /* CT_SAMPLE_*                             */
    double theta_step;          /* mixed sampling only                     */
    uint64_t seed;
} ct_sched_params;

typedef struct ct_schedule ct_schedule;

/* Flat view of a schedule: epoch e uses cols[epoch_col_ptr[e] ..
 * epoch_col_ptr[e+1]); column entry c has groups [col_group_ptr[c],
 * col_group_ptr[c+1]); group g has row blocks rbs[group_rb_ptr[g] ..
 * group_rb_ptr[g+1]) and relaxation beta[g]. */
typedef struct ct_sched_view {
    int32_t n_epochs, n_cols, n_groups, n_rbs;
    const int32_t* epoch_col_ptr;
    const int32_t* cols;
    const int32_t* col_group_ptr;
    const int32_t* group_rb_ptr;
    const int32_t* rbs;
    const double* beta;
} ct_sched_view;

/* nnz: host [m][n] block densities (e.g. from ct_geom_block_nnz). */
int ct_schedule_create(const ct_geom* geom, const ct_sched_params* params, const int64_t* nnz,
                       ct_schedule** out);
/* As ct_schedule_create with any nonnegative block density weights w[m*n]
 * (e.g. ct_geom_block_area): P(I,J) = w / sum_I w, summed in ascending I. */
int ct_schedule_create_w(const ct_geom* geom, const ct_sched_params* params, const double* w,
                         ct_schedule** out);
/* Import an explicit schedule (host arrays, copied).  Each column block may
 * appear at most once per epoch and the row blocks of one column entry must
 * be distinct. */
int ct_schedule_import(const ct_geom* geom, const ct_sched_view* view, ct_schedule** out);
/* Pointers stay valid until ct_schedule_destroy. */
int ct_schedule_export(const ct_schedule* sched, ct_sched_view* out);
void ct_schedule_destroy(ct_schedule* sched);

/* ---- solver state and epochs (Alg. 4 / 5 / 6) ------------------------------ */
enum { CT_SYNC_COLUMN = 0, CT_SYNC_EPOCH = 1 };

typedef struct ct_solver_params {
    int32_t sync;               /* CT_SYNC_COLUMN: r refreshed after every
                                   column block (the listings); CT_SYNC_EPOCH:
                                   all column blocks read the epoch-start r */
} ct_solver_params;

typedef struct ct_solver ct_solver;

/* Device workspace (bytes, 256-aligned) a solver needs for this geometry:
 * the partial projections z^j of every column block (Alg. 4), the residual
 * r, and the per-group buffers of one column-block step (the group
 * gradients g_J, A g and the float64 partial sums of Eq. 11). */
int ct_solver_workspace_bytes(const ct_geom* geom, const ct_solver_params* params,
                              size_t* bytes);
/* workspace: caller-owned device buffer of at least that many bytes, kept
 * alive for the solver's lifetime.  The geometry must outlive the solver. */
int ct_solver_create(ct_geom* geom, const ct_solver_params* params, void* workspace,
                     size_t ws_bytes, ct_solver** out);
void ct_solver_destroy(ct_solver* solver);
/* Start state of Alg. 4: with x == NULL, z^j = 0 and r = y (x must then be
 * zero); otherwise z^j = A^j x_J and r = y - sum_j z^j.  Must be called
 * before the first ct_block_epoch of a solver. */
int ct_solver_reset(ct_solver* solver, const float* y, const float* x, void* stream);
/* One epoch `epoch` of the schedule, updating x (device, [N]) in place. */
int ct_block_epoch(ct_solver* solver, const ct_schedule* sched, int32_t epoch, const float* y,
                   float* x, void* stream);
/* Device pointers into the solver workspace: z [n][M], r [M].  Between
 * epochs a solver's whole state is x, z and r: every other workspace buffer
 * is written within each step before it is read, or holds zeros.  Copying
 * x, z and r out after an epoch and back into a solver of the same geometry
 * and sync mode (after its ct_solver_reset) checkpoints the run; the resumed
 * epochs repeat the uninterrupted run's bit for bit. */
int ct_solver_state(const ct_solver* solver, float** z, float** r);
/* ||y - A x||_2 / ||y||_2 with a full forward projection (reading C16);
 * synchronous on `stream`. */
int ct_true_residual(ct_solver* solver, const float* y, const float* x, double* rel,
                     void* stream);
/* Asynchronous form for convergence checks that must not stall the stream:
 * out (device, 2 doubles) receives ||y - A x||^2 and ||y||^2, each a
 * fixed-order float64 sum.  Uses the solver's scratch (do not overlap with
 * an epoch of the same solver on another stream). */
int ct_residual_norms(ct_solver* solver, const float* y, const float* x, double* out,
                      void* stream);

/* Kernel timing: while enabled, every kernel a solver enqueues is bracketed
 * by HIP events on its stream (a small per-launch cost).  Reading syncs those
 * events and returns, per kernel class, the summed device time (ms) and the
 * launch count since the last read; reading resets the counters. */
enum { CT_K_BACK = 0, CT_K_FWD = 1, CT_K_STEP = 2, CT_K_FINALIZE = 3, CT_K_RESIDUAL = 4,
       CT_K_COUNT = 5 };
typedef struct ct_kernel_times {
    double ms[8];
    int64_t launches[8];
} ct_kernel_times;
int ct_solver_profile(ct_solver* solver, int32_t enable);
int ct_solver_profile_read(ct_solver* solver, ct_kernel_times* out);

/* ---- whole solve ----------------------------------------------------------- */
typedef struct ct_solve_params {
    ct_sched_params sched;      /* sched.epochs = epoch cap               */
    ct_solver_params solver;
    double tau;                 /* nnz threshold (mm)                      */
    double rel_tol;             /* stop when true residual <= rel_tol      */
    int32_t check_every;        /* epochs between residual checks (0: never) */
} ct_solve_params;

typedef struct ct_solve_stats {
    int32_t epochs_run;
    double rel_residual;        /* last checked true relative residual    */
    int64_t ray_voxel_updates;  /* 2 * sum over groups of nnz(A_{I_G}^J)  */
    double* r_norm;             /* in: host array of params->sched.epochs
                                   doubles, or NULL; out: ||r||_2 of the
                                   tracked residual after each epoch run   */
} ct_solve_stats;

/* The whole iteration of Alg. 4-6: the density table (Sec. II-C), the
 * schedule drawn from it (Alg. 5/6), then epochs from x = 0, z^j = 0, r = y
 * until the cap or, every check_every epochs, until the true relative
 * residual ||y - A x|| / ||y|| (reading C16: the tracked r of Sec. II-B is an
 * approximation) is <= rel_tol.  x: device [N], overwritten.  workspace:
 * caller-owned device memory of ct_solver_workspace_bytes(geom,
 * &params->solver) bytes, 256-byte aligned, not retained after the call.
 * The schedule's device tables and, on first use, the geometry's are
 * allocated by the library.  stats may be NULL.  Returns CT_NOT_CONVERGED if
 * the cap was reached before rel_tol (with check_every > 0), CT_EINVAL for a
 * bad argument or a short workspace (nothing enqueued).  Synchronous. */
int ct_solve(ct_geom* geom, const ct_solve_params* params, const float* y, float* x,
             void* workspace, size_t ws_bytes, ct_solve_stats* stats, void* stream);

/* ---- batched epochs --------------------------------------------------------
 * Many independent jobs (each its own geometry, solver, schedule, y and x)
 * advanced together, for workloads of many small reconstructions.  One batch
 * epoch runs the next epoch of Alg. 6 of every job that has one left: for
 * each step index c, ONE launch per projector kind does the back-projection
 * of step c of every job, then one launch the forward projections, one the
 * step sizes and one the finalize; epoch-synchronous jobs then get their
 * residual refresh, and a last tiny launch moves every job's epoch counter
 * on.  Each work-group finds its job in a device job table, so a job's
 * results are bit for bit those of ct_block_epoch run alone.
 *
 * Jobs are added and removed between batch epochs (continuous batching); the
 * batch only refers to the caller's solvers, schedules and buffers, which must
 * outlive the job's membership.  A job's solver must have been reset
 * (ct_solver_reset) and belongs to one batch job at a time; no two jobs may
 * share a solver or an x.  All calls on one batch must use the same stream
 * (or be ordered by the caller): the job table is updated on that stream. */
typedef struct ct_batch ct_batch;
typedef struct ct_batch_job {
    ct_solver* solver;
    const ct_schedule* sched;   /* built for the solver's geometry          */
    const float* y;             /* device [M]                               */
    float* x;                   /* device [N], updated in place             */
    int32_t epoch;              /* first epoch of sched to run              */
} ct_batch_job;
/* CT_BATCH_GRAPH: record the launches of one batch epoch into a HIP graph
 * once (again after every add/remove) and replay it; the kernels read each
 * job's epoch from the device, so one graph serves every epoch. */
enum { CT_BATCH_GRAPH = 1 };
/* capacity: most jobs the batch holds at once (1..256). */
int ct_batch_create(int32_t capacity, ct_batch** out);
void ct_batch_destroy(ct_batch* batch);
/* Adds a job; *id identifies it until ct_batch_remove. */
int ct_batch_add(ct_batch* batch, const ct_batch_job* job, int32_t* id);
int ct_batch_remove(ct_batch* batch, int32_t id);
/* One batch epoch; *ran (may be NULL) = jobs that had an epoch to run. */
int ct_batch_epoch(ct_batch* batch, int32_t flags, int32_t* ran, void* stream);
/* Next epoch the job will run (== its schedule's epoch count when done). */
int ct_batch_job_epoch(const ct_batch* batch, int32_t id, int32_t* epoch);
/* Kernel timing of the batched launches, as ct_solver_profile (the phase
 * launches are timed per kernel class; while enabled, CT_BATCH_GRAPH is
 * ignored and the launches go out one by one). */
int ct_batch_profile(ct_batch* batch, int32_t enable);
int ct_batch_profile_read(ct_batch* batch, ct_kernel_times* out);

/* ---- launch shapes and their tuner ------------------------------------------
 * Two launch-shape choices of the projectors leave what is computed unchanged
 * (only the order of float32 sums moves): how many pieces each chord of the
 * fused forward pass is walked in (fwd_split: 1, 2 or 4 waves per 64 rays),
 * and how many waves share the views of a 2D back-projection tile
 * (back_waves: 1, 2, 4, 8 or 16; the 3D tile always takes 4).  They are not steps
 * of the method: they serve the batched and served system patterns, whose
 * jobs range from small slices to large volumes.  Default: 4 and 4.
 *
 * ct_geom_tune times every shape as whole epochs of a scratch solver on the
 * schedule's first epoch (zero data: the projectors do the same work), keeps
 * the fastest for the geometry, and caches the table of times per (geometry
 * kind, voxels per column block and rays per row block rounded to powers of
 * two, GPU architecture), so later geometries of that size class are not
 * timed again.  It allocates scratch device memory (a solver workspace, y
 * and x) for the length of the call and synchronises the stream.  Calls that
 * use the geometry must not run meanwhile.  Errors: CT_EINVAL (NULL, unknown
 * flags, a schedule of another geometry, a shape outside the sets above),
 * CT_EDEVICE. */
typedef struct ct_tuning {
    int32_t fwd_split;
    int32_t back_waves;
    double ms;                  /* tuner: mean epoch time of the chosen shape */
    double ms_default;          /* tuner: the same for the default shape */
    int32_t trials;             /* shapes timed by this call (0: from the cache) */
    int32_t cached;             /* 1: the times came from the cache */
} ct_tuning;

enum { CT_TUNE_REFRESH = 1 };   /* time again even if the size class is cached */

/* Set / read the shapes a geometry's launches use (solver steps and the
 * back-projection primitive). */
int ct_geom_set_tuning(ct_geom* geom, const ct_tuning* t);
int ct_geom_get_tuning(const ct_geom* geom, ct_tuning* t);
int ct_geom_tune(ct_geom* geom, const ct_schedule* sched, int32_t flags, ct_tuning* out,
                 void* stream);

/* For each geometry kind among a batch's jobs, the shape whose epoch times
 * summed over those jobs (each from its size class, timed as above if not
 * cached) are smallest.  The jobs' geometries take it too, so that a job run
 * alone reproduces its batch results bit for bit.  out: ct_tuning[4] indexed
 * by kind (zeros for kinds no job has), may be NULL.  The batch's captured
 * graph is dropped (the shapes are part of it). */
int ct_batch_tune(ct_batch* batch, int32_t flags, ct_tuning* out, void* stream);
/* Set the shapes of one kind's batched launches (the jobs' geometries are not
 * changed). */
int ct_batch_set_tuning(ct_batch* batch, int32_t kind, const ct_tuning* t);

/* ---- serving ---------------------------------------------------------------
 * A request loop over a batch (continuous batching): jobs are submitted with
 * their geometry, schedule parameters and measurements, wait in a FIFO queue,
 * and enter the batch at a tick boundary when a slot is free and their device
 * footprint fits the HBM budget.  While resident, a job's geometry tables,
 * y, x and z^j stay on the device; every tick runs one batch epoch for all
 * resident jobs, and every check_every epochs (and at the epoch cap) a job's
 * true relative residual is computed asynchronously and read back at the next
 * tick, which retires the job once it is <= rel_tol or the cap is reached.
 * A retired job's x is copied to the host and its device memory reused.  The
 * server allocates its device memory once, when it is created: an arena of
 * the budget, sub-allocated per job, and a pinned host staging ring (a
 * quarter of the budget, 64 MiB .. 1 GiB) for every copy between host and
 * device; a tick allocates and frees nothing and waits for the device only
 * for the residual norms of the previous tick.  A job's density table is
 * counted on the device when it is admitted and read back asynchronously, so
 * it joins the batch's epochs from a later tick.  All ticks of a server must
 * use the same stream. */
typedef struct ct_server ct_server;
typedef struct ct_server_params {
    int32_t capacity;           /* most resident jobs (1..256)                  */
    int64_t hbm_budget;         /* device bytes resident jobs may use; 0 = 80% of
                                   free memory when the server is created      */
    double rel_tol;             /* retire at true relative residual <= rel_tol  */
    int32_t check_every;        /* epochs between residual checks (>= 1)        */
    double tau;                 /* nnz threshold of the density table (mm)      */
    int32_t use_graph;          /* replay batch epochs from a HIP graph         */
} ct_server_params;
typedef struct ct_server_job {
    const ct_geom_desc* geom;   /* copied at submit                             */
    ct_sched_params sched;      /* sched.epochs = epoch cap                     */
    ct_solver_params solver;
    const float* y;             /* host [M], copied at submit                   */
    int64_t tag;                /* caller's label, returned with the result     */
} ct_server_job;
typedef struct ct_server_done {
    int64_t tag;
    int32_t id;
    int32_t status;             /* CT_OK: converged; CT_NOT_CONVERGED: cap; <0 error */
    int32_t epochs;             /* epochs run                                   */
    double rel_residual;        /* last checked true relative residual          */
    double t_submit, t_admit, t_done;   /* seconds on the server's clock        */
    int64_t bytes;              /* device bytes charged to the budget           */
    int64_t updates;            /* ray-voxel updates of its epochs (2 nnz per
                                   group update)                                */
} ct_server_done;
typedef struct ct_server_stats {
    int32_t active, queued;
    int64_t admitted, retired;
    int64_t updates;            /* ray-voxel updates of all epochs run so far   */
    int64_t bytes_in_use, budget;
    double now;                 /* server clock (s)                             */
} ct_server_stats;
int ct_server_create(const ct_server_params* params, ct_server** out);
void ct_server_destroy(ct_server* server);
/* Queues a job (its geometry is validated and its host tables built here);
 * CT_EINVAL if the geometry is invalid or the job can never fit the budget or
 * the staging ring. */
int ct_server_submit(ct_server* server, const ct_server_job* job, int32_t* id);
/* Retire finished jobs, admit queued ones, run one batch epoch. */
int ct_server_tick(ct_server* server, void* stream, ct_server_stats* stats);
/* Up to max finished jobs (oldest first), removed from the server's list. */
int ct_server_poll(ct_server* server, ct_server_done* out, int32_t max, int32_t* n);
/* x (host, [N]) of a finished job; each result can be taken once. */
int ct_server_result(ct_server* server, int32_t id, float* x);

/* Device bytes one job needs (geometry tables + workspace): for admission
 * by memory budget. */
int ct_job_footprint(const ct_geom_desc* desc, const ct_solver_params* params, size_t* bytes);

const char* ct_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CT_H */
