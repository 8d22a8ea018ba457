// Host-callable launchers of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bsgd_device.h"

namespace bsgd {

// Per-iteration schedule record, int32, `stride` entries:
//   [0]                    number of views in this iteration
//   [1, 1+R)               selected row blocks (ascending)
//   [1+R, 2+2R)            offsets of each selected row block's views into the view list
//   [2+2R, 2+2R+B)         selected column blocks (ascending)
//   [2+2R+B, +maxv)        view list (row blocks in order, views ascending in each)
//   [2+2R+B+maxv, +2)      iteration counter k (low, high 32 bits)
struct SchedLayout {
    int32_t R, B, maxv, stride;
    __host__ __device__ int off_rows() const { return 1; }
    __host__ __device__ int off_gstart() const { return 1 + R; }
    __host__ __device__ int off_blocks() const { return 2 + 2 * R; }
    __host__ __device__ int off_views() const { return 2 + 2 * R + B; }
    __host__ __device__ int off_k() const { return 2 + 2 * R + B + maxv; }
    static __host__ __device__ int stride_for(int R, int B, int maxv) { return 4 + 2 * R + B + maxv; }
};

// Draws: int8 per (iteration, view slot, block slot); -1 = skip view, >= 0 sub-detector.
constexpr int8_t DRAW_SKIP = -1;

// Maximum column blocks per geometry (the residual kernels stage one view's
// footprint rectangles in LDS).
constexpr int MAX_BLOCKS = 1024;
// Largest views-per-workgroup of the LDS-staged forward projector.
constexpr int FP_CHUNK_MAX = 16;

// One solve of a batched launch (device array). base[p] is the entry's first
// workgroup in the batched grid of phase p (0 forward projection, 1 residual,
// 2 back projection + step); gx[p] its workgroups along x (the per-solve grid's
// y extent is B, maxv, B).
struct BatchEntry {
    DevGeom G;
    SchedLayout L;
    const int32_t* sched;  // schedule records of this call
    const PairWork* work;  // work records of this call
    const float* y;
    float* x;
    float* xT;             // copy of x stored y fastest (global-memory walk), or NULL
    float* z;
    float* ghat;
    float* gsum;
    float* r_sel;          // 2D: {w2, slope, lmax, r} per selected ray; 3D: r
    const float* mu;  // device scalar (the current step length)
    int fp_chunk;
    int fp_lds;
    long long n_vox;
    int gx[3];
    int base[3];
};

// Per-solve grid of each phase (x extent, total workgroups) for a batch entry.
void batch_grids(BatchEntry& e);

// Entries of one batched launch group, passed by value as the kernel argument (the
// 4 KB argument segment holds up to BATCH_GROUP entries): pointers read from kernel
// arguments are known to address global memory, so the shared bodies compile to the
// same global (not flat) loads and scalar loads as in the single-solve kernels.
constexpr int BATCH_GROUP = 12;
struct BatchArgs {
    BatchEntry e[BATCH_GROUP];
    int n;    // entries in use
    int it;   // iteration index into every entry's records
    int id0;  // workgroup id of this launch's first workgroup (forward and 2D back projection classes)
};
static_assert(sizeof(BatchArgs) <= 4096, "batched kernel arguments must fit the 4 KB argument segment");

// A contiguous range of phase-0 workgroups whose entries share one LDS size.
struct FpLaunchClass {
    int wg0, wgs;
    size_t lds_bytes;
};
// A contiguous range of back-projection workgroups whose solves share the 2D wave split.
struct BpLaunchClass {
    int wg0, wgs, split;
};
// Launch one iteration (A.it) of all entries of A; the entries share the dimension;
// wgs[p] = total workgroups of phase p over the group.
hipError_t launch_batch_iteration(BatchArgs& A, int dim, const int (&wgs)[3], const FpLaunchClass* fp_classes,
                                  int n_fp_classes, const BpLaunchClass* bp_classes, int n_bp_classes,
                                  size_t res_lds_bytes, hipStream_t st);
size_t fp_lds_bytes_for(const DevGeom& G);
size_t resid_lds_bytes_for(const DevGeom& G);

hipError_t launch_geom_stats(const DevGeom& G, double* w, int64_t* nnz, hipStream_t st);

// Draws (when q != NULL) and per-(block slot, view slot) work records for n_iters
// iterations: draws [n][maxv][B] (may be NULL), work [n][B][maxv]. The iteration
// counter of each record is read from the schedule.
hipError_t launch_plan(const DevGeom& G, const int32_t* sched, SchedLayout L, int n_iters, uint64_t seed,
                       const uint32_t* q, int64_t im_until, int8_t* draws, PairWork* work, hipStream_t st);

// blocks_sel: the iteration's selected blocks (device, inside its schedule record).
// xT: the copy of x stored y fastest ([z][x][y]) for the global-memory walk, or NULL.
hipError_t launch_fp_pairs(const DevGeom& G, const PairWork* work_it, SchedLayout L, const int32_t* blocks_sel,
                           const float* x, const float* xT, float* z, hipStream_t st);

hipError_t launch_resid(const DevGeom& G, const int32_t* sched_it, SchedLayout L, const float* y,
                        const float* z, float* r_sel, hipStream_t st);

// delta == NULL: per-row-block memories ghat (Algorithm 1); else the sub-detector memory
// form, reading the residual changes `delta` (z layout) and leaving ghat alone.
// xT (or NULL): the copy of x stored y fastest, kept equal to x for the voxels updated.
hipError_t launch_bp_step(const DevGeom& G, const int32_t* sched_it, const PairWork* work_it, SchedLayout L,
                          const float* r_sel, const float* delta, float* ghat, float* gsum, float* x, float* xT,
                          const float* mu, int64_t n_vox, hipStream_t st);
// xT[(z nx + x) ny + y] = x[(z ny + y) nx + x]: the copy of x stored y fastest.
hipError_t launch_xy_transpose(const float* x, float* xT, int nx, int ny, int nz, hipStream_t st);

// delta = r - rho and rho = r over every selected pair's pixel range (z layout).
hipError_t launch_subdet_delta(const DevGeom& G, const int32_t* sched_it, const PairWork* work_it, SchedLayout L,
                               const float* r_sel, float* rho, float* delta, hipStream_t st);

// Standalone projectors over a device view list (views[n_sel]); block < 0 = all blocks.
hipError_t launch_fp_full(const DevGeom& G, const int32_t* views, int n_sel, int block, const float* x,
                          float* y, int accumulate, hipStream_t st);
hipError_t launch_bp_full(const DevGeom& G, const int32_t* views, int n_sel, int block, const float* y,
                          float* x, float scale, int accumulate, hipStream_t st);

// ||y - sum_j z^j||^2 over all rays into partials; returns number of partials written.
hipError_t launch_resid_sumsq(const DevGeom& G, const float* y, const float* z, double* partials,
                              int* n_partials, hipStream_t st);
// sum of squares of a float array into partials.
hipError_t launch_sumsq(const float* a, int64_t n, double* partials, int* n_partials, hipStream_t st);
// out[0] = sum of partials[0..n) in index order.
hipError_t launch_sum_partials(const double* partials, int n, double* out, hipStream_t st);

// a[i] = b[i] - c[i]
hipError_t launch_sub(const float* b, const float* c, float* a, int64_t n, hipStream_t st);
hipError_t launch_fill(float* a, float v, int64_t n, hipStream_t st);
// a[i] += b[i]
hipError_t launch_add(float* a, const float* b, int64_t n, hipStream_t st);
// partial sums of a . b (FP64) into partials
hipError_t launch_dot(const float* a, const float* b, int64_t n, double* partials, int* n_partials, hipStream_t st);

// TV proximal step of BSGD-TV on x (in place): iters fast-gradient-projection steps.
// wstep: device {w, step} (prox weight w = mu lambda and the dual step 1/(4 dim w),
// written by tv_weight_step), read by the kernels at run time so that captured graphs
// see step-length changes. p, ra, rb: device [dim][n_vox] scratch each, holding the
// last three dual iterates in rotation.
hipError_t launch_tv_prox(const DevGeom& G, float* x, const float* wstep, int iters, float* p, float* ra,
                          float* rb, hipStream_t st);
// Bounds of the pixel rectangle (columns, rows) one 3D back-projection workgroup tile
// projects to in any view, from the geometry (DevGeom::bp3_kmax, bp3_lmax); 0 when
// staging in LDS is off (then every view reads global memory).
void set_bp3_bounds(DevGeom& G, double sod, double sdd, double du, double dv);
// Host values of {w, step} for step length mu and TV weight lambda.
void tv_weight_step(int dim, double mu, double lambda, float* out);

}  // namespace bsgd
