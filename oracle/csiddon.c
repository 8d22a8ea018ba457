/*
 * Plain FP64 matrix-free Siddon projector: y = A x and g = A^T r.
 *
 * TEST INFRASTRUCTURE (oracle). Used by the tests to build or apply A on grids
 * too large for the pure-Python Siddon, and timed as the CPU baseline. It
 * restates the same definition as oracle/siddon.py (Sec. I after Eq. (yax):
 * a_ij = length of ray i inside voxel j, Siddon / Jacobs et al. 1998): the ray is
 * p0 + alpha (p1 - p0); the alpha values of the grid planes inside the grid are
 * merged in increasing order (each axis' planes are already monotone in alpha);
 * each pair of consecutive values bounds a segment whose voxel is the floor of
 * its midpoint and whose length is the alpha difference times |p1 - p0|.
 * Zero-length segments are dropped; an axis with zero direction contributes no
 * planes and requires the ray to lie in that slab (half-open voxels).
 *
 * Pinned against oracle/siddon.py on small grids (tests).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int dim;
    int64_t n[3];
    double lo[3];
    double v[3];
} grid_t;

/* Visit every segment of one ray; emit(voxel, length, ctx). Returns segment count. */
typedef void (*emit_fn)(int64_t voxel, double len, void *ctx);

static int64_t walk_ray(const grid_t *g, const double *p0, const double *p1, emit_fn emit, void *ctx)
{
    double d[3] = {0, 0, 0}, L2 = 0.0;
    int dim = g->dim;
    for (int a = 0; a < dim; ++a) {
        d[a] = p1[a] - p0[a];
        L2 += d[a] * d[a];
    }
    double len = sqrt(L2);
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < dim; ++a) {
        double lo = g->lo[a], hi = g->lo[a] + (double)g->n[a] * g->v[a];
        if (d[a] != 0.0) {
            double a0 = (lo - p0[a]) / d[a], a1 = (hi - p0[a]) / d[a];
            double mn = a0 < a1 ? a0 : a1, mx = a0 < a1 ? a1 : a0;
            if (mn > amin) amin = mn;
            if (mx < amax) amax = mx;
        } else if (!(lo <= p0[a] && p0[a] < hi)) {
            return 0;
        }
    }
    if (!(amin < amax)) return 0;

    /* next plane index and step per axis, in increasing alpha */
    int64_t next[3] = {0, 0, 0}, step[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        if (d[a] > 0.0) {
            step[a] = 1;
            next[a] = 0;
        } else if (d[a] < 0.0) {
            step[a] = -1;
            next[a] = g->n[a];
        }
    }
    /* skip planes at or before amin */
    double na[3];
    for (int a = 0; a < dim; ++a) {
        na[a] = INFINITY;
        if (step[a] == 0) continue;
        for (;;) {
            if (next[a] < 0 || next[a] > g->n[a]) break;
            double al = (g->lo[a] + (double)next[a] * g->v[a] - p0[a]) / d[a];
            if (al > amin) {
                na[a] = al;
                break;
            }
            next[a] += step[a];
        }
    }
    double cur = amin;
    int64_t count = 0;
    for (;;) {
        double nxt = amax;
        int which = -1;
        for (int a = 0; a < dim; ++a) {
            if (na[a] < nxt) {
                nxt = na[a];
                which = a;
            }
        }
        if (nxt > cur) {
            double mid = 0.5 * (cur + nxt);
            int64_t flat = 0, stride = 1;
            for (int a = 0; a < dim; ++a) {
                double c = p0[a] + mid * d[a];
                int64_t i = (int64_t)floor((c - g->lo[a]) / g->v[a]);
                if (i < 0) i = 0;
                if (i > g->n[a] - 1) i = g->n[a] - 1;
                flat += i * stride;
                stride *= g->n[a];
            }
            emit(flat, (nxt - cur) * len, ctx);
            ++count;
        }
        if (which < 0) break;
        cur = nxt;
        next[which] += step[which];
        if (next[which] < 0 || next[which] > g->n[which]) {
            na[which] = INFINITY;
        } else {
            double al = (g->lo[which] + (double)next[which] * g->v[which] - p0[which]) / d[which];
            na[which] = al < amax ? al : INFINITY;
        }
    }
    return count;
}

static void make_grid(grid_t *g, int dim, const int64_t *n, const double *lo, const double *v)
{
    g->dim = dim;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = a < dim ? n[a] : 1;
        g->lo[a] = a < dim ? lo[a] : 0.0;
        g->v[a] = a < dim ? v[a] : 1.0;
    }
}

typedef struct { const double *x; double acc; int64_t nnz; } fp_ctx;
static void fp_emit(int64_t vox, double len, void *c)
{
    fp_ctx *f = (fp_ctx *)c;
    f->acc += len * f->x[vox];
    f->nnz += 1;
}

typedef struct { double *g; double r; } bp_ctx;
static void bp_emit(int64_t vox, double len, void *c)
{
    bp_ctx *b = (bp_ctx *)c;
    b->g[vox] += len * b->r;
}

typedef struct { int64_t *idx; double *val; int64_t n, cap; } row_ctx;
static void row_emit(int64_t vox, double len, void *c)
{
    row_ctx *r = (row_ctx *)c;
    if (r->n < r->cap) {
        r->idx[r->n] = vox;
        r->val[r->n] = len;
    }
    r->n += 1;
}

/* y[i] = sum_j a_ij x_j for each ray; returns total nonzeros visited. */
int64_t oracle_fp(int dim, const int64_t *n, const double *lo, const double *v, int64_t n_rays,
                  const double *p0, const double *p1, const double *x, double *y, int n_threads)
{
    grid_t g;
    make_grid(&g, dim, n, lo, v);
    int64_t total = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
#endif
    for (int64_t i = 0; i < n_rays; ++i) {
        fp_ctx c = {x, 0.0, 0};
        walk_ray(&g, p0 + i * dim, p1 + i * dim, fp_emit, &c);
        y[i] = c.acc;
        total += c.nnz;
    }
    return total;
}

/* out[j] = sum_i a_ij r_i; per-thread private accumulators summed in thread order. */
void oracle_bp(int dim, const int64_t *n, const double *lo, const double *v, int64_t n_rays,
               const double *p0, const double *p1, const double *r, double *out, int n_threads)
{
    grid_t g;
    make_grid(&g, dim, n, lo, v);
    int64_t c = g.n[0] * g.n[1] * g.n[2];
    memset(out, 0, sizeof(double) * (size_t)c);
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    if (nt <= 1) {
        bp_ctx b = {out, 0.0};
        for (int64_t i = 0; i < n_rays; ++i) {
            if (r[i] == 0.0) continue;
            b.r = r[i];
            walk_ray(&g, p0 + i * dim, p1 + i * dim, bp_emit, &b);
        }
        return;
    }
    double *priv = (double *)calloc((size_t)nt * (size_t)c, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        bp_ctx b = {priv + (size_t)t * (size_t)c, 0.0};
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n_rays; ++i) {
            if (r[i] == 0.0) continue;
            b.r = r[i];
            walk_ray(&g, p0 + i * dim, p1 + i * dim, bp_emit, &b);
        }
    }
#endif
    for (int t = 0; t < nt; ++t)
        for (int64_t j = 0; j < c; ++j) out[j] += priv[(size_t)t * (size_t)c + j];
    free(priv);
}

/* Segments of one ray; returns the count (entries beyond cap are not written). */
int64_t oracle_ray(int dim, const int64_t *n, const double *lo, const double *v, const double *p0,
                   const double *p1, int64_t *idx, double *val, int64_t cap)
{
    grid_t g;
    make_grid(&g, dim, n, lo, v);
    row_ctx r = {idx, val, 0, cap};
    walk_ray(&g, p0, p1, row_emit, &r);
    return r.n;
}

/* Count nonzeros per ray (for CSR row pointers). */
void oracle_count(int dim, const int64_t *n, const double *lo, const double *v, int64_t n_rays,
                  const double *p0, const double *p1, int64_t *counts, int n_threads)
{
    grid_t g;
    make_grid(&g, dim, n, lo, v);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n_rays; ++i) {
        row_ctx r = {NULL, NULL, 0, 0};
        walk_ray(&g, p0 + i * dim, p1 + i * dim, row_emit, &r);
        counts[i] = r.n;
    }
}

/* Fill CSR (indices, data) given row pointers from oracle_count. */
void oracle_fill(int dim, const int64_t *n, const double *lo, const double *v, int64_t n_rays,
                 const double *p0, const double *p1, const int64_t *indptr, int64_t *indices,
                 double *data, int n_threads)
{
    grid_t g;
    make_grid(&g, dim, n, lo, v);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n_rays; ++i) {
        row_ctx r = {indices + indptr[i], data + indptr[i], 0, indptr[i + 1] - indptr[i]};
        walk_ray(&g, p0 + i * dim, p1 + i * dim, row_emit, &r);
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
