/*
 * bsgd.h - C ABI of the MI355X block stochastic gradient descent (BSGD) library.
 *
 * The operations follow Gao, Biguri, Blumensath, "Block stochastic gradient
 * descent for large-scale tomographic reconstruction in a parallel network":
 *
 *   y = A x + e,  min_x 1/2 ||y - A x||^2                     (Sec. I, Eqs. (yax), (min))
 *   a_ij = length of ray i inside voxel j (Siddon)              (Sec. I, after Eq. (yax))
 *   A is never stored; A x and A^T r are computed on the fly    (Sec. I)
 *   A partitioned into M row blocks I_i and N column blocks J_j (Sec. II, Eq. (e1))
 *   BSGD / BSGD-IM / BSGD-TV iterations                         (Algorithms 1, 2, 4)
 *   alpha, gamma from the node count                            (Eq. 1)
 *
 * Conventions shared by every call
 * --------------------------------
 * Units are millimetres; A's entries are lengths in mm. Device arrays are FP32.
 * The volume is centred at the origin, voxel (i,j,k) centred at
 * ((i-(nx-1)/2) vx, (j-(ny-1)/2) vy, (k-(nz-1)/2) vz), stored [z][y][x] (x fastest).
 * View m has angle angles_rad[m]; the source is at sod (cos t, sin t, 0), the flat
 * detector is centred at -(sdd-sod)(cos t, sin t, 0) with u-axis (-sin t, cos t, 0)
 * and v-axis (0,0,1); pixel (k,l) is centred at u=(k-(nu-1)/2)du, v=(l-(nv-1)/2)dv.
 * Parallel beam (2D) ray k passes through u_k (-sin t, cos t) along (cos t, sin t).
 * Projections are stored [view][v][u] (u fastest). 2D kinds need nz = nv = 1.
 * Column block j = (tz by + ty) bx + tx covers the tile [floor(t n/b), floor((t+1) n/b))
 * along each axis. Row blocks are groups of whole views: a permutation of the views
 * drawn from partition_seed is cut into M consecutive groups (the first n_views mod M
 * one view longer), views ascending within a group.
 *
 * Ownership: the caller owns every pointer it passes (device pointers for x, y, r;
 * host pointers where stated) and the stream; the library owns geometry tables and
 * solver state, allocates them through the geometry's allocator (bsgd_allocator;
 * hipMalloc when none is given) and frees them in *_destroy.
 * Calls are asynchronous on the given stream (a hipStream_t, NULL = default stream)
 * unless they return host values, which synchronise that stream.
 * Errors: every call returns a status; no exception crosses the ABI. Invalid
 * arguments return BSGD_E_INVALID_ARG before any device work is enqueued.
 * bsgd_last_error() gives a thread-local message for the last non-OK status.
 * Thread safety: distinct objects may be used from distinct threads; one object
 * must not be used concurrently.
 */
#ifndef BSGD_H
#define BSGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSGD_OK = 0,
    BSGD_E_INVALID_ARG = 1,
    BSGD_E_UNSUPPORTED = 2,
    BSGD_E_OUT_OF_MEMORY = 3,
    BSGD_E_DEVICE = 4,
    BSGD_E_DIVERGED = 5,
    BSGD_E_STATE = 6
} bsgd_status;

typedef enum { BSGD_PARALLEL_2D = 0, BSGD_FAN_FLAT_2D = 1, BSGD_CONE_FLAT_3D = 2 } bsgd_kind;

/* Sub-detector sampling of Algorithm 2 (BSGD-IM, Fig. 2).
 * NONE    : plain BSGD, every ray of the selected views is used.
 * COLNORM : probability of sub-detector s for (view v, block j) proportional to
 *           ||A[rows of s in v, J_j]||_F^2 (the denser sub-matrix is the likelier,
 *           Sec. II-A), quantised to integers q = round(2^20 w / sum w) (>= 1 if w > 0).
 * AREA    : proportional to the area of block j's projection (the shadow of its
 *           corners, in detector pixel units, pixel k spanning [k - 1/2, k + 1/2])
 *           that falls on sub-detector s: the estimate of the sub-matrix density the
 *           paper gives for Algorithm 2 (Sec. II-A); same quantisation. In 2D the shadow
 *           is an interval and the area its length.
 * UNIFORM : every sub-detector equally likely (BSGD-RAN, Sec. III-E-3). */
typedef enum { BSGD_IM_NONE = 0, BSGD_IM_COLNORM = 1, BSGD_IM_AREA = 2, BSGD_IM_UNIFORM = 3 } bsgd_im_mode;

/* Device memory provider for a geometry and every solver created from it (for example
 * a framework's caching allocator). alloc returns `bytes` of device memory usable on
 * `stream` (NULL on failure); free releases a pointer alloc returned, on the stream it
 * was allocated for. ctx and both functions must stay valid until the geometry and its
 * solvers are destroyed. */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, void* stream);
} bsgd_allocator;

typedef struct {
    int32_t kind;                 /* bsgd_kind */
    int32_t nx, ny, nz;           /* voxels per axis (nz = 1 in 2D) */
    double vx, vy, vz;            /* voxel size, mm */
    int32_t n_views;
    const double* angles_rad;     /* host [n_views], copied */
    int32_t nu, nv;               /* detector pixels (nv = 1 in 2D) */
    double du, dv;                /* detector pitch, mm */
    double sod, sdd;              /* source-to-centre, source-to-detector, mm (fan/cone) */
    int32_t bx, by, bz;           /* column-block tiling, N = bx by bz <= 1024 (bz = 1 in 2D) */
    int32_t n_row_blocks;         /* M */
    uint64_t partition_seed;      /* seed of the view-to-row-block permutation */
    int32_t su, sv;               /* sub-detectors per view (IM), S = su sv <= 16 */
    int32_t im_mode;              /* bsgd_im_mode */
    const uint32_t* im_table;     /* optional host [n_views][S][N] sampling weights; NULL = computed */
    const bsgd_allocator* allocator; /* device memory of tables and solver state; NULL = hipMalloc
                                        (the struct is copied, its ctx and functions are kept) */
} bsgd_geometry_desc;

typedef struct bsgd_geometry bsgd_geometry;
typedef struct bsgd_solver bsgd_solver;

/* The system matrix A of Sec. I (a_ij = length of ray i inside voxel j, never stored)
 * and its partition of Sec. II, Eq. (e1): M row blocks of whole views and N column
 * blocks of the image, with the sampling tables of Algorithm 2. Validates the
 * descriptor, builds the partitions, the per-(view, block) detector footprints, the
 * projected areas of the AREA mode and, on the device, the per-(view, sub-detector,
 * block) squared norms and nonzero counts of A (computed for every mode). Synchronises
 * `stream`. Invalid descriptors (an unknown kind or sampling mode, sizes out of range,
 * a volume not strictly between source and detector, an allocator without both
 * functions) return BSGD_E_INVALID_ARG before any device work; *out is NULL on any
 * failure. */
bsgd_status bsgd_geometry_create(const bsgd_geometry_desc* desc, void* stream, bsgd_geometry** out);
void bsgd_geometry_destroy(bsgd_geometry* geom);

typedef struct {
    int64_t n_rays;          /* n_views nv nu */
    int64_t n_voxels;        /* nx ny nz */
    int32_t n_blocks;        /* N */
    int32_t n_row_blocks;    /* M */
    int32_t n_subdet;        /* S */
    int32_t max_group_views; /* views in the largest row block */
    int64_t z_floats;        /* floats of compact z storage (sum of footprint areas) */
    int64_t nnz;             /* nonzeros of A (segments of positive FP32 length) */
} bsgd_geometry_info;

bsgd_status bsgd_geometry_get_info(const bsgd_geometry* geom, bsgd_geometry_info* out);

/* Host copies of geometry tables (out must hold `bytes`):
 * VIEW_ORDER  int32 [n_views]          views of row block 0, then 1, ... (ascending in a group)
 * GROUP_START int32 [M + 1]            offsets of each row block into VIEW_ORDER
 * IM_WEIGHTS  double [n_views][S][N]   ||A[rows of sub-detector s of view v, J_j]||_F^2
 * IM_TABLE    uint32 [n_views][S][N]   quantised sampling table in use
 * NNZ         int64 [n_views][S][N]    nonzeros of each such sub-matrix
 * FOOTPRINT   int32 [n_views][N][4]    detector rectangle [u0, u1) x [v0, v1) of block j
 * IM_AREA     double [n_views][S][N]   area of block j's projection on sub-detector s (pixels^2) */
typedef enum {
    BSGD_TABLE_VIEW_ORDER = 0,
    BSGD_TABLE_GROUP_START = 1,
    BSGD_TABLE_IM_WEIGHTS = 2,
    BSGD_TABLE_IM_TABLE = 3,
    BSGD_TABLE_NNZ = 4,
    BSGD_TABLE_FOOTPRINT = 5,
    BSGD_TABLE_IM_AREA = 6
} bsgd_table;
bsgd_status bsgd_geometry_table(const bsgd_geometry* geom, int32_t which, void* out, size_t bytes);

/* Launch-shape tuning of a geometry. fp_views_per_group: views whose rays one
 * workgroup of the LDS-staged forward projector walks, in [1, 16] (default 12); it
 * does not change any result. fp_ray_split: lanes that share one ray of a 2D forward
 * projection through a block, 1, 2 or 4 (default 1): the chord is cut into that many
 * equal parameter segments, walked in parallel and summed in a fixed order, so
 * results depend on it only through FP32 rounding and are reproducible for a given
 * value (3D rays are never split). fp_waves_per_pair: waves of the global-memory
 * forward walk (blocks too large for the LDS stage) per (view, block) pair, in [1, 64]
 * (default from the mean footprint); it does not change any result; 0 in
 * bsgd_geometry_set_tuning keeps the current value. fp_staged (filled by
 * bsgd_geometry_get_tuning, ignored by set): 1 when the forward projector stages
 * blocks in LDS (fp_views_per_group and fp_ray_split apply), 0 when it walks global
 * memory (fp_waves_per_pair applies). bp_waves: waves of a 2D back-projection
 * workgroup, 2, 4 or 8 (default 4): each wave gathers a share of the views into the
 * tile's voxels and the shares are added in a fixed order, so results depend on it only
 * through FP32 rounding and are reproducible for a given value; 0 in
 * bsgd_geometry_set_tuning keeps the current value; 3D geometries ignore it. Solvers
 * read the shape at each launch; a solver that already captured its epoch graph keeps
 * the shape it captured. reserved must be 0. */
typedef struct {
    int32_t fp_views_per_group;
    int32_t fp_ray_split;
    int32_t fp_waves_per_pair;
    int32_t fp_staged;
    int32_t bp_waves;
    int32_t reserved[3];
} bsgd_tuning;
bsgd_status bsgd_geometry_set_tuning(bsgd_geometry* geom, const bsgd_tuning* tuning);
bsgd_status bsgd_geometry_get_tuning(const bsgd_geometry* geom, bsgd_tuning* tuning);

#define BSGD_ACCUMULATE 1u

/* Forward projection (Sec. I: FP = A x):
 *   y[a][l][k] (= or +=) sum_{j in blocks} (A_{views[a]}^{J_j} x_{J_j})[l][k]
 * x: device [nz][ny][nx]; y: device [n_sel][nv][nu] with n_sel = n_views_sel, or
 * all views in index order when views == NULL. views: host int32 list (copied).
 * block = -1 projects the whole volume, otherwise only column block `block`.
 * flags: BSGD_ACCUMULATE adds into y instead of overwriting. A non-NULL views list with
 * n_views_sel = 0 selects no view: nothing is written and y may be NULL. */
bsgd_status bsgd_forward_project(const bsgd_geometry* geom, const float* x, float* y,
                                 const int32_t* views, int32_t n_views_sel, int32_t block,
                                 uint32_t flags, void* stream);

/* Matched back projection (Sec. I: BP = A^T r), same lengths as the forward projection:
 *   x[J] (= or +=) scale * (A_{views}^{J})^T y
 * for every voxel of `block` (all voxels when block = -1); voxels outside J are untouched.
 * y: device [n_sel][nv][nu] as for bsgd_forward_project. With an empty views list
 * (n_views_sel = 0, y may be NULL) the sum is empty: x[J] is set to 0, or left as it is
 * with BSGD_ACCUMULATE. */
bsgd_status bsgd_back_project(const bsgd_geometry* geom, const float* y, float* x,
                              const int32_t* views, int32_t n_views_sel, int32_t block,
                              float scale, uint32_t flags, void* stream);

/* Solver options.
 * rows_per_iter, blocks_per_iter: alpha M and gamma N of Algorithm 1. If both are 0,
 *   node_count P gives them through Eq. 1: gamma = min(1, P/N), alpha = P/(M N gamma)
 *   (non-integer results are rejected).
 * mu: the paper's step length; the update is g = 2 A^T r, x += mu g (Eq. (SGDITE)).
 * seed: selection and importance-sampling streams. Every draw is a pure function of
 *   (seed, stream, counters): SplitMix64 output function, keys folded one by one.
 * tv_lambda > 0 enables Algorithm 4: every tv_every iterations (0 = round(1/(alpha gamma)))
 *   x <- argmin_t ||t - x||^2 + 2 mu lambda TV(t) by tv_inner_iters fast-gradient-projection
 *   steps (isotropic TV, backward differences, zero difference across the low boundary).
 * max_effective_epochs, tol: bsgd_solve stops after max_effective_epochs effective epochs
 *   (one epoch = round(1/(alpha gamma)) iterations), or earlier when tol > 0 and the
 *   relative normal-equation residual ||A^T(y - A x)|| / ||A^T y|| <= tol, checked
 *   every check_every epochs (0 = every epoch).
 * flags: BSGD_FLAG_EAGER, BSGD_FLAG_SUBDET_MEMORY (below); other bits are rejected.
 * auto_mu: Algorithm 3 (Sec. II-A). Every M iterations the g of the last M iterations
 *   are summed into an effective update direction (EUD), theta is the cosine of two
 *   consecutive EUDs and ||r|| = ||y - sum_j z^j||; once three norms and two thetas
 *   exist: three decreasing norms -> mu *= 1 + eps; three increasing norms and
 *   (|theta - theta_prev| > t1 or theta < t2) -> mu *= 1 - delta. Costs one
 *   synchronisation every M iterations; not available in bsgd_step_batch.
 * im_until: with importance sampling (Algorithm 2), only iterations k < im_until draw
 *   sub-detectors; iterations k >= im_until use every ray of the selected row blocks
 *   (plain Algorithm 1), the unbiased tail Sec. II-A recommends for the last iterations
 *   (sampled g_hat entries bias the fixed point; the plain tail converges to the
 *   least-squares solution). 0 = sample in every iteration. */
typedef struct {
    int32_t rows_per_iter;
    int32_t blocks_per_iter;
    int32_t node_count;
    int32_t tv_inner_iters;
    double mu;
    uint64_t seed;
    double tv_lambda;
    int32_t tv_every;
    int32_t max_effective_epochs;
    double tol;
    int32_t check_every;
    int32_t flags;                /* BSGD_FLAG_* */
    int32_t auto_mu;              /* 1: automatic step length (Algorithm 3) */
    int32_t im_until;             /* first iteration without importance sampling; 0 = none */
    double mu_eps, mu_delta;      /* Algorithm 3 epsilon, delta; 0 = 0.05, 0.4 */
    double mu_t1, mu_t2;          /* Algorithm 3 thresholds t1, t2; 0 = 0.1, 0.5 */
} bsgd_options;

/* Launch every kernel directly instead of replaying a captured HIP graph of one
 * effective epoch (graphs are used when a bsgd_step call covers whole epochs from an
 * epoch boundary and per-kernel profiling is off). Results are identical. */
#define BSGD_FLAG_EAGER 1

/* Keep the gradient memory per (view, sub-detector, column block) instead of per
 * (row block, column block) (the unbiased form of Algorithm 2, Sec. II-A). A pair
 * refreshes the memories of the (view, sub-detector) parts whose rays it used, and
 * g is the sum of all memories; without importance sampling the iterates equal
 * Algorithm 1's (a row block's part memories sum to its g_hat). With sampling, a
 * drawn sub-detector no longer stands for its whole view, so at a fixed point g is
 * the full gradient 2 A^T (y - A x) and the iteration reaches the least-squares
 * solution. Stored as each ray's residual at its last refresh (z layout, z_floats
 * floats, plus as many for the changes) instead of the M x c floats of g_hat.
 * Not available in bsgd_step_batch. */
#define BSGD_FLAG_SUBDET_MEMORY 2

/* Create a solver for y (device [n_views][nv][nu], must stay valid and unchanged while
 * the solver lives) and x (device [nz][ny][nx], the initial image, updated in place by
 * bsgd_step). State z = 0, g_hat = 0, g = 0 (Algorithm 1, initialisation). */
bsgd_status bsgd_solver_create(const bsgd_geometry* geom, const float* y, float* x,
                               const bsgd_options* opt, void* stream, bsgd_solver** out);

/* Run n_iters iterations of Algorithm 1/2/4 on the solver's stream. If resid_norm_out
 * is not NULL, synchronise and return ||y - sum_j z^j|| (the maintained residual r of
 * Algorithm 1); a non-finite value returns BSGD_E_DIVERGED. */
bsgd_status bsgd_step(bsgd_solver* s, int32_t n_iters, double* resid_norm_out);

/* Run n_iters iterations of every solver in solvers[0..n) with one launch per phase
 * (forward projection, residual rebuild, back projection + step) covering all of
 * them: the batched, continuous-serving form of bsgd_step. Each solve's arithmetic is
 * the same as in bsgd_step (same kernels, same per-workgroup decomposition), so its
 * iterates are bitwise identical alone and in any batch. All solvers must have been
 * created on `stream`, share the dimension (2D or 3D) and be distinct. Asynchronous.
 * Errors mark every solver of the batch as failed. */
bsgd_status bsgd_step_batch(bsgd_solver* const* solvers, int32_t n, int32_t n_iters, void* stream);

/* Stopping statistic of bsgd_solve for several solves at once: out[i] =
 * ||A^T (y - A x_i)|| of solver i's current image (the normal-equation residual; the
 * least-squares problem of Sec. I is solved where it vanishes), divided by
 * ||A^T y|| when `relative` is non-zero (computed on the first relative call and
 * kept). Everything is enqueued on `stream` (every solver must have been created on
 * it) and the call synchronises once. Each solver allocates n_rays + n_voxels floats
 * of scratch on its first call. out is host memory of n doubles. */
bsgd_status bsgd_normal_residual(bsgd_solver* const* solvers, int32_t n, int32_t relative, double* out,
                                 void* stream);

/* Allocation-free form of bsgd_normal_residual (relative = 0) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc. *out = ||A^T (y - A x)|| for the geometry's whole
 * system, y device [n_views][nv][nu], x device [nz][ny][nx] (caller owned, read only),
 * out host. The same kernels as bsgd_normal_residual, so the same value bit for bit.
 * Scratch (the residual, its back projection, reduction partials) lives in one static
 * device array of bsgd_noalloc_scratch_bytes() bytes (64 MiB) per GPU, held until the
 * process ends; a geometry needing more (about 4 (n_rays + n_voxels) bytes + 33 KB)
 * returns BSGD_E_INVALID_ARG before any device work. No hipMalloc, hipFree or other
 * allocation. Calls on one GPU share that array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * Synchronises `stream` once. */
bsgd_status bsgd_normal_residual_noalloc(const bsgd_geometry* geom, const float* y, const float* x, double* out,
                                         void* stream);
size_t bsgd_noalloc_scratch_bytes(void);

/* Asynchronous form of bsgd_normal_residual for serving loops that must not wait on
 * the device: enqueues, for every solver i, ||A^T (y - A x_i)||^2 into out_sq[2 i] and
 * ||A^T y||^2 into out_sq[2 i + 1] (computed on the solver's first call and kept on the
 * device), copied to host memory out_sq (page-locked for the copy to be asynchronous)
 * in stream order; out_sq is valid once `stream` has passed this call (an event or a
 * synchronisation). Same kernels and values as bsgd_normal_residual. */
bsgd_status bsgd_normal_residual_async(bsgd_solver* const* solvers, int32_t n, double* out_sq, void* stream);

/* Current step length and its value after each Algorithm 3 check (history[0..cap)). */
bsgd_status bsgd_solver_step_length(const bsgd_solver* s, double* mu_now, double* history, int32_t cap,
                                    int32_t* n_history);

/* Iterations done so far, and alpha M, gamma N, iterations per effective epoch. */
bsgd_status bsgd_solver_counts(const bsgd_solver* s, int64_t* iters_done, int32_t* rows_per_iter,
                               int32_t* blocks_per_iter, int32_t* epoch_iters);

/* Host copy of the schedule of the last bsgd_step call (synchronises):
 * rows [n][rows_per_iter], blocks [n][blocks_per_iter] (ascending), and the drawn
 * sub-detectors draws [n][max_group_views * rows_per_iter][blocks_per_iter]
 * (int16; view slot order = row blocks in `rows` order, views ascending in each;
 * -1 = view skipped, -2 = no sampling). Any output may be NULL. n = iterations of that call. */
bsgd_status bsgd_solver_last_schedule(const bsgd_solver* s, int32_t* n_out, int32_t* rows,
                                      int32_t* blocks, int16_t* draws, size_t draws_bytes);

/* Copy solver state to caller device memory: which = 0 g [c], 1 g_hat [M][c], 2 z (compact,
 * z_floats), 3 the residual snapshots of BSGD_FLAG_SUBDET_MEMORY (z layout, z_floats; the
 * memory of (view, sub-detector, block) is 2 (A_part^J)^T of its part of them). Asking for
 * g_hat with that flag, or for 3 without it, is BSGD_E_INVALID_ARG. */
bsgd_status bsgd_solver_state(const bsgd_solver* s, int32_t which, float* out, size_t bytes);

/* Per-kernel time accounting with HIP events on the solver's stream (off by default).
 * kernel ids: 0 forward projection, 1 residual rebuild, 2 back projection + step,
 * 3 TV prox, 4 sampling draws. ms_out[5] total milliseconds, launches_out[5] counts. */
bsgd_status bsgd_solver_set_profiling(bsgd_solver* s, int32_t on);
bsgd_status bsgd_solver_kernel_times(bsgd_solver* s, double* ms_out, int64_t* launches_out);

void bsgd_solver_destroy(bsgd_solver* s);

/* The reconstruction of Sec. I, min 1/2 ||y - A x||^2, by Algorithms 1, 2 and 4 (the
 * options select the form): create a solver for (y, x), step whole effective epochs
 * until the stopping rule of bsgd_options (tol, max_effective_epochs), write the image
 * to x, destroy the solver. x holds the initial image on entry. *iters_out and
 * *resid_norm_out (either may be NULL) receive the iterations run and ||y - sum_j z^j||.
 * Synchronises `stream`. Errors as bsgd_solver_create and bsgd_step; x then holds the
 * last iterate reached. */
bsgd_status bsgd_solve(const bsgd_geometry* geom, const float* y, float* x, const bsgd_options* opt,
                       void* stream, int32_t* iters_out, double* resid_norm_out);

const char* bsgd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSGD_H */
