// Host runtime and C ABI of the BSGD library: geometry tables (partitions,
// detector footprints, block-local ray anchors, importance-sampling tables),
// solver state, the per-iteration schedule and kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsgd.h"
#include "bsgd_device.h"
#include "bsgd_kernels.h"

using namespace bsgd;

// ------------------------------------------------------------ errors

static thread_local std::string g_err;

static bsgd_status fail(bsgd_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(e_ == hipErrorOutOfMemory ? BSGD_E_OUT_OF_MEMORY : BSGD_E_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                              \
    } while (0)

extern "C" const char* bsgd_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------ counter-based streams (host)

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr uint64_t STREAM_PARTITION = 1, STREAM_ROWS = 2, STREAM_BLOCKS = 3;

uint64_t mix64h(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t hash_keys(uint64_t seed, uint64_t stream, std::initializer_list<uint64_t> keys)
{
    uint64_t h = mix64h(seed + GOLDEN * (1 + stream));
    for (uint64_t k : keys) h = mix64h(h ^ k);
    return h;
}

uint64_t bounded(uint64_t h, uint64_t n) { return (uint64_t)(((unsigned __int128)h * n) >> 64); }

// m distinct indices of [0, n) for iteration k: partial Fisher-Yates, then ascending.
void choose(uint64_t seed, uint64_t stream, int64_t k, int n, int m, int32_t* out, std::vector<int32_t>& scratch)
{
    scratch.resize(n);
    for (int i = 0; i < n; ++i) scratch[i] = i;
    for (int t = 0; t < m; ++t) {
        int jj = t + (int)bounded(hash_keys(seed, stream, {(uint64_t)k, (uint64_t)t}), (uint64_t)(n - t));
        std::swap(scratch[t], scratch[jj]);
    }
    std::sort(scratch.begin(), scratch.begin() + m);
    std::copy(scratch.begin(), scratch.begin() + m, out);
}

// Device buffer from the geometry's allocator (hipMalloc when there is none), released
// on the stream it was allocated for.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    const bsgd_allocator* A = nullptr;
    hipStream_t st = nullptr;
    ~DevBuf() { release(); }
    void use(const bsgd_allocator* a, hipStream_t s)
    {
        release();
        A = a;
        st = s;
    }
    void release()
    {
        if (p) {
            if (A)
                A->free(A->ctx, p, (void*)st);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b)
    {
        release();
        if (b == 0) b = 16;
        if (A) {
            p = A->alloc(A->ctx, b, (void*)st);
            if (!p) return hipErrorOutOfMemory;
            bytes = b;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    template <class T>
    T* as() const
    {
        return reinterpret_cast<T*>(p);
    }
};

// Page-locked host blocks, recycled through a process-wide pool instead of being freed
// (freeing page-locked memory waits for the whole device): a block of at least `bytes`
// (sizes rounded up to powers of two, at least 256 bytes).
std::mutex g_pin_mu;
std::vector<std::pair<size_t, void*>> g_pin_free;

size_t pin_class(size_t b)
{
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}

hipError_t pinned_get(void** out, size_t b, size_t* got)
{
    const size_t c = pin_class(b);
    {
        std::lock_guard<std::mutex> lock(g_pin_mu);
        for (size_t i = 0; i < g_pin_free.size(); ++i)
            if (g_pin_free[i].first == c) {
                *out = g_pin_free[i].second;
                g_pin_free.erase(g_pin_free.begin() + i);
                if (got) *got = c;
                return hipSuccess;
            }
    }
    hipError_t e = hipHostMalloc(out, c, hipHostMallocDefault);
    if (e == hipSuccess && got) *got = c;
    return e;
}

void pinned_put(void* p, size_t b)
{
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pin_mu);
    g_pin_free.push_back({pin_class(b), p});
}

// Pinned host staging buffer whose reuse waits for the previous copy out of it.
struct Staging {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    ~Staging()
    {
        if (done) {
            if (pending) (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        pinned_put(host, bytes);
    }
    hipError_t reserve(size_t b)
    {
        if (!done) {
            hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (pending) {
            hipError_t e = hipEventSynchronize(done);
            if (e != hipSuccess) return e;
            pending = false;
        }
        if (b <= bytes) return hipSuccess;
        pinned_put(host, bytes);
        host = nullptr;
        bytes = 0;
        size_t got = 0;
        hipError_t e = pinned_get(&host, b, &got);
        if (e == hipSuccess) bytes = got;
        return e;
    }
    hipError_t upload(void* dst, size_t b, hipStream_t st)
    {
        hipError_t e = hipMemcpyAsync(dst, host, b, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        e = hipEventRecord(done, st);
        pending = (e == hipSuccess);
        return e;
    }
};

}  // namespace

// ------------------------------------------------------------ geometry

struct bsgd_geometry {
    bsgd_geometry_desc d{};
    std::vector<double> angles;
    int dim = 2, N = 1, M = 1, S = 1, max_group = 1;
    int64_t n_rays = 0, n_vox = 0, z_floats = 0, nnz_total = 0;
    std::vector<int32_t> view_order, group_start;
    std::vector<PairInfo> pairs;
    std::vector<BlockInfo> blocks;
    std::vector<double> im_w;
    std::vector<int64_t> im_nnz;
    std::vector<uint32_t> im_q;
    std::vector<float4> raydir, raynorm, raytrap;
    std::vector<float2> rayv;
    std::vector<float> kspan;
    std::vector<double> im_area;  // projected area of block j on sub-detector s of view v
    DevBuf d_cs, d_pairs, d_blocks, d_q, d_all_views, d_views, d_raydir, d_rayv, d_raynorm, d_raytrap, d_kspan;
    DevBuf d_cov_off, d_cov_idx;
    Staging stage;
    DevGeom dg{};
    bsgd_allocator alloc_copy{};
    const bsgd_allocator* alloc = nullptr;  // &alloc_copy when the descriptor gave one
    hipStream_t st = nullptr;               // stream the tables were allocated on
    void bind(DevBuf& b) const { b.use(alloc, st); }
    void bind_all()
    {
        for (DevBuf* b : {&d_cs, &d_pairs, &d_blocks, &d_q, &d_all_views, &d_views, &d_raydir, &d_rayv, &d_raynorm,
                          &d_raytrap, &d_kspan, &d_cov_off, &d_cov_idx})
            bind(*b);
    }
};

static bsgd_status validate(const bsgd_geometry_desc* d)
{
    if (!d) return fail(BSGD_E_INVALID_ARG, "descriptor is NULL");
    if (d->kind < 0 || d->kind > 2) return fail(BSGD_E_INVALID_ARG, "unknown geometry kind %d", d->kind);
    const bool is3d = d->kind == BSGD_CONE_FLAT_3D;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(BSGD_E_INVALID_ARG, "grid sizes must be >= 1");
    if (!is3d && (d->nz != 1 || d->nv != 1 || d->bz != 1 || d->sv != 1))
        return fail(BSGD_E_INVALID_ARG, "2D geometries need nz = nv = bz = sv = 1");
    if (!(d->vx > 0 && d->vy > 0 && d->vz > 0) || !std::isfinite(d->vx) || !std::isfinite(d->vy) ||
        !std::isfinite(d->vz))
        return fail(BSGD_E_INVALID_ARG, "voxel sizes must be positive and finite");
    if (d->n_views < 1 || d->n_views > 65535) return fail(BSGD_E_INVALID_ARG, "n_views must be in [1, 65535]");
    if (!d->angles_rad) return fail(BSGD_E_INVALID_ARG, "angles_rad is NULL");
    for (int m = 0; m < d->n_views; ++m)
        if (!std::isfinite(d->angles_rad[m])) return fail(BSGD_E_INVALID_ARG, "angle %d is not finite", m);
    if (d->nu < 1 || d->nv < 1) return fail(BSGD_E_INVALID_ARG, "detector sizes must be >= 1");
    if ((int64_t)d->nu * d->nv > (int64_t)1 << 30) return fail(BSGD_E_INVALID_ARG, "detector too large");
    if (!(d->du > 0 && d->dv > 0) || !std::isfinite(d->du) || !std::isfinite(d->dv))
        return fail(BSGD_E_INVALID_ARG, "detector pitch must be positive and finite");
    if ((int64_t)d->nx * d->ny * d->nz > ((int64_t)1 << 31) - 1) return fail(BSGD_E_INVALID_ARG, "volume too large");
    if (d->bx < 1 || d->by < 1 || d->bz < 1 || d->bx > d->nx || d->by > d->ny || d->bz > d->nz)
        return fail(BSGD_E_INVALID_ARG, "block tiling must satisfy 1 <= b <= n per axis");
    if ((int64_t)d->bx * d->by * d->bz > MAX_BLOCKS)
        return fail(BSGD_E_INVALID_ARG, "at most %d column blocks", MAX_BLOCKS);
    if (d->n_row_blocks < 1 || d->n_row_blocks > d->n_views)
        return fail(BSGD_E_INVALID_ARG, "n_row_blocks must be in [1, n_views]");
    if (d->su < 1 || d->sv < 1 || d->su > d->nu || d->sv > d->nv || d->su * d->sv > 16)
        return fail(BSGD_E_INVALID_ARG, "sub-detectors: 1 <= su <= nu, 1 <= sv <= nv, su sv <= 16");
    if (d->im_mode != BSGD_IM_NONE && d->im_mode != BSGD_IM_COLNORM && d->im_mode != BSGD_IM_AREA &&
        d->im_mode != BSGD_IM_UNIFORM)
        return fail(BSGD_E_INVALID_ARG, "unknown im_mode %d", d->im_mode);
    if (d->allocator && (!d->allocator->alloc || !d->allocator->free))
        return fail(BSGD_E_INVALID_ARG, "an allocator needs both alloc and free");
    if (d->kind != BSGD_PARALLEL_2D) {
        if (!(d->sod > 0 && d->sdd > d->sod) || !std::isfinite(d->sdd))
            return fail(BSGD_E_INVALID_ARG, "need 0 < sod < sdd");
        const double rx = 0.5 * d->nx * d->vx, ry = 0.5 * d->ny * d->vy;
        const double R = std::sqrt(rx * rx + ry * ry);
        if (!(R < d->sod) || !(R < d->sdd - d->sod))
            return fail(BSGD_E_INVALID_ARG, "the volume must lie strictly between source and detector");
    }
    return BSGD_OK;
}

static void tile(int n, int b, int t, int& lo, int& hi)
{
    lo = (int)(((int64_t)t * n) / b);
    hi = (int)(((int64_t)(t + 1) * n) / b);
}

static void build_tables(bsgd_geometry* g)
{
    const bsgd_geometry_desc& d = g->d;
    const bool is3d = d.kind == BSGD_CONE_FLAT_3D;
    const bool par = d.kind == BSGD_PARALLEL_2D;
    g->dim = is3d ? 3 : 2;
    g->N = d.bx * d.by * d.bz;
    g->M = d.n_row_blocks;
    g->S = d.su * d.sv;
    g->n_rays = (int64_t)d.n_views * d.nu * d.nv;
    g->n_vox = (int64_t)d.nx * d.ny * d.nz;

    // row blocks: seeded Fisher-Yates permutation cut into M consecutive groups
    std::vector<int32_t> perm(d.n_views);
    for (int i = 0; i < d.n_views; ++i) perm[i] = i;
    for (int t = 0; t + 1 < d.n_views; ++t) {
        int jj = t + (int)bounded(hash_keys(d.partition_seed, STREAM_PARTITION, {(uint64_t)t}),
                                  (uint64_t)(d.n_views - t));
        std::swap(perm[t], perm[jj]);
    }
    const int base = d.n_views / g->M, extra = d.n_views % g->M;
    g->view_order.clear();
    g->group_start.assign(1, 0);
    int pos = 0;
    g->max_group = 0;
    for (int i = 0; i < g->M; ++i) {
        int size = base + (i < extra ? 1 : 0);
        std::vector<int32_t> grp(perm.begin() + pos, perm.begin() + pos + size);
        std::sort(grp.begin(), grp.end());
        g->view_order.insert(g->view_order.end(), grp.begin(), grp.end());
        pos += size;
        g->group_start.push_back(pos);
        g->max_group = std::max(g->max_group, size);
    }

    // column blocks
    const double lox = -0.5 * d.nx * d.vx, loy = -0.5 * d.ny * d.vy, loz = -0.5 * d.nz * d.vz;
    g->blocks.resize(g->N);
    std::vector<double> cbx(g->N), cby(g->N), cbz(g->N), ex0(g->N), ex1(g->N), ey0(g->N), ey1(g->N), ez0(g->N),
        ez1(g->N);
    for (int tz = 0; tz < d.bz; ++tz)
        for (int ty = 0; ty < d.by; ++ty)
            for (int tx = 0; tx < d.bx; ++tx) {
                const int j = (tz * d.by + ty) * d.bx + tx;
                int x0, x1, y0, y1, z0, z1;
                tile(d.nx, d.bx, tx, x0, x1);
                tile(d.ny, d.by, ty, y0, y1);
                tile(d.nz, d.bz, tz, z0, z1);
                BlockInfo& B = g->blocks[j];
                std::memset(&B, 0, sizeof B);
                B.x0 = x0;
                B.y0 = y0;
                B.z0 = z0;
                B.nbx = x1 - x0;
                B.nby = y1 - y0;
                B.nbz = z1 - z0;
                B.hx = (float)(0.5 * B.nbx * d.vx);
                B.hy = (float)(0.5 * B.nby * d.vy);
                B.hz = (float)(0.5 * B.nbz * d.vz);
                ex0[j] = lox + x0 * d.vx;
                ex1[j] = lox + x1 * d.vx;
                ey0[j] = loy + y0 * d.vy;
                ey1[j] = loy + y1 * d.vy;
                ez0[j] = loz + z0 * d.vz;
                ez1[j] = loz + z1 * d.vz;
                cbx[j] = 0.5 * (ex0[j] + ex1[j]);
                cby[j] = 0.5 * (ey0[j] + ey1[j]);
                cbz[j] = 0.5 * (ez0[j] + ez1[j]);
            }

    // per (view, block): detector footprint and block-local ray anchors
    const double ku = 0.5 * (d.nu - 1), lv = 0.5 * (d.nv - 1);
    const double margin = 1e-3;
    g->pairs.resize((size_t)d.n_views * g->N);
    int64_t zoff = 0;
    for (int v = 0; v < d.n_views; ++v) {
        const double c = std::cos(d.angles_rad[v]), s = std::sin(d.angles_rad[v]);
        for (int j = 0; j < g->N; ++j) {
            PairInfo& P = g->pairs[(size_t)v * g->N + j];
            std::memset(&P, 0, sizeof P);
            double kmin = INFINITY, kmax = -INFINITY, lmin = INFINITY, lmax = -INFINITY;
            for (int q = 0; q < 8; ++q) {
                const double X = (q & 1) ? ex1[j] : ex0[j];
                const double Y = (q & 2) ? ey1[j] : ey0[j];
                const double Z = (q & 4) ? ez1[j] : ez0[j];
                const double w = -X * s + Y * c;
                double kk, ll = 0.0;
                if (par) {
                    kk = w / d.du + ku;
                } else {
                    const double dep = d.sod - (X * c + Y * s);
                    kk = d.sdd * w / dep / d.du + ku;
                    if (is3d) ll = d.sdd * Z / dep / d.dv + lv;
                }
                kmin = std::min(kmin, kk);
                kmax = std::max(kmax, kk);
                lmin = std::min(lmin, ll);
                lmax = std::max(lmax, ll);
            }
            int u0 = (int)std::max(0.0, std::ceil(kmin - margin));
            int u1 = (int)std::min((double)d.nu, std::floor(kmax + margin) + 1.0);
            int v0 = 0, v1 = 1;
            if (is3d) {
                v0 = (int)std::max(0.0, std::ceil(lmin - margin));
                v1 = (int)std::min((double)d.nv, std::floor(lmax + margin) + 1.0);
            }
            if (u1 <= u0 || v1 <= v0) u0 = u1 = v0 = v1 = 0;
            P.u0 = u0;
            P.u1 = u1;
            P.v0 = v0;
            P.v1 = v1;
            P.zoff = zoff;
            zoff += (int64_t)(u1 - u0) * (v1 - v0);

            const double cu = -cbx[j] * s + cby[j] * c;
            const double ce = cbx[j] * c + cby[j] * s;
            P.cu = (float)cu;
            P.cz = (float)cbz[j];
            if (par) {
                const int kc = (int)std::lround(cu / d.du + ku);
                P.kc = kc;
                P.au = (float)d.du;
                P.bu = (float)((kc - ku) * d.du - cu);
                P.depth = 0.0f;
            } else {
                const double D = d.sod - ce;
                const double A = D / d.sdd;
                const int kc = (int)std::lround(cu / A / d.du + ku);
                P.kc = kc;
                P.au = (float)(A * d.du);
                P.bu = (float)(A * (kc - ku) * d.du - cu);
                P.depth = (float)D;
                if (is3d) {
                    const int lc = (int)std::lround(cbz[j] / A / d.dv + lv);
                    P.lc = lc;
                    P.av = (float)(A * d.dv);
                    P.bv = (float)(A * (lc - lv) * d.dv - cbz[j]);
                }
            }
        }
    }
    g->z_floats = zoff;

    // ray tables: reciprocal direction components and lengths, FP64 rounded once
    auto recip = [](double a) { return a == 0.0 ? INFINITY : (float)(1.0 / a); };
    g->raydir.resize((size_t)d.n_views * d.nu);
    for (int v = 0; v < d.n_views; ++v) {
        const double c = std::cos(d.angles_rad[v]), s = std::sin(d.angles_rad[v]);
        for (int k = 0; k < d.nu; ++k) {
            float4 T;
            if (par) {
                T = make_float4(recip(c), recip(s), 1.0f, 0.0f);
            } else {
                const double u = (k - ku) * d.du;
                const double a = -d.sdd * c - u * s, b = -d.sdd * s + u * c;
                const double n2 = d.sdd * d.sdd + u * u;
                T = make_float4(recip(a), recip(b), is3d ? (float)n2 : (float)std::sqrt(n2), 0.0f);
            }
            g->raydir[(size_t)v * d.nu + k] = T;
        }
    }
    g->rayv.resize(d.nv);
    for (int l = 0; l < d.nv; ++l) {
        const double vv = (l - lv) * d.dv;
        g->rayv[l] = make_float2(recip(vv), (float)(vv * vv));
    }

    // 2D chord tables: unit normal of each ray, xi (n . p = lambda xi for the anchor
    // point p = lambda e_u), and the chord trapezoid through one voxel
    if (!is3d) {
        const double hx = 0.5 * d.vx, hy = 0.5 * d.vy;
        g->raynorm.resize((size_t)d.n_views * d.nu);
        g->raytrap.resize((size_t)d.n_views * d.nu);
        g->kspan.resize(2 * (size_t)d.n_views);
        for (int v = 0; v < d.n_views; ++v) {
            const double c = std::cos(d.angles_rad[v]), s = std::sin(d.angles_rad[v]);
            double span = 0.0, span2 = 0.0;
            for (int k = 0; k < d.nu; ++k) {
                double nx, ny, xi, len;
                if (par) {
                    nx = -s;
                    ny = c;
                    xi = 1.0;
                    len = 1.0;
                } else {
                    const double u = (k - ku) * d.du;
                    const double a = -d.sdd * c - u * s, b = -d.sdd * s + u * c;
                    len = std::sqrt(d.sdd * d.sdd + u * u);
                    nx = -b / len;
                    ny = a / len;
                    xi = -d.sdd / len;
                }
                const double ax = std::fabs(nx), ay = std::fabs(ny);
                const double w2 = hx * ax + hy * ay, w1 = std::fabs(hx * ax - hy * ay);
                const double lx = ay > 0 ? d.vx / ay : INFINITY, ly = ax > 0 ? d.vy / ax : INFINITY;
                const double lmax = std::min(lx, ly);
                // an axis-aligned ray has a box profile (w1 = w2): a huge finite slope
                // gives the same chord and keeps (w2 - |delta|) * slope free of inf * 0
                const double slope = w2 > w1 ? std::min(lmax / (w2 - w1), 1e30) : 1e30;
                g->raynorm[(size_t)v * d.nu + k] = make_float4((float)nx, (float)ny, (float)xi, 0.0f);
                g->raytrap[(size_t)v * d.nu + k] = make_float4((float)w1, (float)w2, (float)lmax, (float)slope);
                span = std::max(span, w2 * len / d.du);
                // two x-adjacent voxels as one 2 x 1 rectangle: support half-width 2 hx |nx| + hy |ny|
                span2 = std::max(span2, (w2 + hx * ax) * len / d.du);
            }
            g->kspan[v] = (float)(span * (1.0 + 1e-5));
            g->kspan[(size_t)d.n_views + v] = (float)(span2 * (1.0 + 1e-5));
        }
    }
}

// Pixel-major index of z (DevGeom::cov_off / cov_idx): for every ray, the z slots of the
// column blocks whose footprint holds its pixel, blocks ascending. Built per view from
// the footprint rectangles (counting, prefix sum, fill) and uploaded view by view.
static bsgd_status upload_cover_index(bsgd_geometry* g, hipStream_t st)
{
    const bsgd_geometry_desc& d = g->d;
    if (g->z_floats >= ((int64_t)1 << 32)) return BSGD_OK;  // rectangle tests instead
    const int64_t per_view = (int64_t)d.nu * d.nv;
    const int64_t n_rays = per_view * d.n_views;
    HIP_TRY(g->d_cov_off.alloc((size_t)(n_rays + 1) * sizeof(uint32_t)));
    HIP_TRY(g->d_cov_idx.alloc((size_t)std::max<int64_t>(g->z_floats, 1) * sizeof(uint32_t)));
    std::vector<uint32_t> off((size_t)per_view + 1), fill((size_t)per_view), idx;
    uint32_t base = 0;
    for (int v = 0; v < d.n_views; ++v) {
        std::fill(off.begin(), off.end(), 0u);
        const PairInfo* pv = g->pairs.data() + (size_t)v * g->N;
        for (int j = 0; j < g->N; ++j)
            for (int l = pv[j].v0; l < pv[j].v1; ++l)
                for (int k = pv[j].u0; k < pv[j].u1; ++k) off[(size_t)l * d.nu + k + 1] += 1;
        off[0] = base;
        for (int64_t q = 0; q < per_view; ++q) off[q + 1] += off[q];
        const uint32_t n_v = off[per_view] - base;
        idx.resize(std::max<uint32_t>(n_v, 1));
        for (int64_t q = 0; q < per_view; ++q) fill[q] = off[q] - base;
        for (int j = 0; j < g->N; ++j) {
            const PairInfo& P = pv[j];
            const int w = P.u1 - P.u0;
            for (int l = P.v0; l < P.v1; ++l)
                for (int k = P.u0; k < P.u1; ++k)
                    idx[fill[(size_t)l * d.nu + k]++] =
                        (uint32_t)(P.zoff + (int64_t)(l - P.v0) * w + (k - P.u0));
        }
        // synchronous copies: the host vectors are reused for the next view
        HIP_TRY(hipMemcpy(g->d_cov_off.as<uint32_t>() + (size_t)v * per_view, off.data(),
                          (size_t)per_view * sizeof(uint32_t), hipMemcpyHostToDevice));
        if (n_v)
            HIP_TRY(hipMemcpy(g->d_cov_idx.as<uint32_t>() + base, idx.data(), (size_t)n_v * sizeof(uint32_t),
                              hipMemcpyHostToDevice));
        base += n_v;
    }
    HIP_TRY(hipMemcpy(g->d_cov_off.as<uint32_t>() + n_rays, &base, sizeof(uint32_t), hipMemcpyHostToDevice));
    if ((int64_t)base != g->z_floats) return fail(BSGD_E_STATE, "z index covers %u of %lld slots", base,
                                                  (long long)g->z_floats);
    (void)st;
    g->dg.cov_off = g->d_cov_off.as<uint32_t>();
    g->dg.cov_idx = g->d_cov_idx.as<uint32_t>();
    return BSGD_OK;
}

static bsgd_status upload_tables(bsgd_geometry* g, hipStream_t st)
{
    const bsgd_geometry_desc& d = g->d;
    std::vector<float2> cs(d.n_views);
    for (int v = 0; v < d.n_views; ++v)
        cs[v] = make_float2((float)std::cos(d.angles_rad[v]), (float)std::sin(d.angles_rad[v]));
    HIP_TRY(g->d_cs.alloc(cs.size() * sizeof(float2)));
    HIP_TRY(g->d_pairs.alloc(g->pairs.size() * sizeof(PairInfo)));
    HIP_TRY(g->d_blocks.alloc(g->blocks.size() * sizeof(BlockInfo)));
    std::vector<int32_t> all(d.n_views);
    for (int v = 0; v < d.n_views; ++v) all[v] = v;
    HIP_TRY(g->d_all_views.alloc(all.size() * sizeof(int32_t)));
    HIP_TRY(g->d_raydir.alloc(g->raydir.size() * sizeof(float4)));
    HIP_TRY(g->d_rayv.alloc(g->rayv.size() * sizeof(float2)));
    HIP_TRY(hipMemcpyAsync(g->d_raydir.p, g->raydir.data(), g->raydir.size() * sizeof(float4), hipMemcpyHostToDevice,
                           st));
    HIP_TRY(hipMemcpyAsync(g->d_rayv.p, g->rayv.data(), g->rayv.size() * sizeof(float2), hipMemcpyHostToDevice, st));
    if (!g->raynorm.empty()) {
        HIP_TRY(g->d_raynorm.alloc(g->raynorm.size() * sizeof(float4)));
        HIP_TRY(g->d_raytrap.alloc(g->raytrap.size() * sizeof(float4)));
        HIP_TRY(g->d_kspan.alloc(g->kspan.size() * sizeof(float)));
        HIP_TRY(hipMemcpyAsync(g->d_raynorm.p, g->raynorm.data(), g->raynorm.size() * sizeof(float4),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(g->d_raytrap.p, g->raytrap.data(), g->raytrap.size() * sizeof(float4),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(g->d_kspan.p, g->kspan.data(), g->kspan.size() * sizeof(float), hipMemcpyHostToDevice,
                               st));
    }
    HIP_TRY(hipMemcpyAsync(g->d_cs.p, cs.data(), cs.size() * sizeof(float2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->d_pairs.p, g->pairs.data(), g->pairs.size() * sizeof(PairInfo), hipMemcpyHostToDevice,
                           st));
    HIP_TRY(hipMemcpyAsync(g->d_blocks.p, g->blocks.data(), g->blocks.size() * sizeof(BlockInfo),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->d_all_views.p, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));

    DevGeom& G = g->dg;
    G.kind = d.kind;
    G.dim = g->dim;
    G.nx = d.nx;
    G.ny = d.ny;
    G.nz = d.nz;
    G.vx = (float)d.vx;
    G.vy = (float)d.vy;
    G.vz = (float)d.vz;
    G.n_views = d.n_views;
    G.nu = d.nu;
    G.nv = d.nv;
    G.du = (float)d.du;
    G.dv = (float)d.dv;
    G.sod = (float)d.sod;
    G.sdd = (float)d.sdd;
    G.N = g->N;
    G.bx = d.bx;
    G.by = d.by;
    G.bz = d.bz;
    G.su = d.su;
    G.sv = d.sv;
    G.S = g->S;
    G.cs = g->d_cs.as<float2>();
    G.pairs = g->d_pairs.as<PairInfo>();
    G.blocks = g->d_blocks.as<BlockInfo>();
    G.raydir = g->d_raydir.as<float4>();
    G.rayv = g->d_rayv.as<float2>();
    G.fp_chunk = 12;
    G.fp_split = 1;
    G.bp_split = 4;  // 2D back projection: views of a voxel over four waves (the measured best on the 512^2 fan)
    // waves per pair of the global-memory forward projector: one per 48 pixels of the
    // mean footprint (about one 64-pixel round per wave; more, shorter waves hide the
    // gather latency of the walk better), at most 64
    {
        double area = 0.0;
        int64_t cnt = 0;
        for (const PairInfo& P : g->pairs)
            if (P.u1 > P.u0 && P.v1 > P.v0) {
                area += (double)(P.u1 - P.u0) * (P.v1 - P.v0);
                ++cnt;
            }
        const double mean = cnt ? area / (double)cnt : 0.0;
        G.fp_wpp = (int)std::min(64.0, std::max(1.0, std::floor(mean / 48.0)));
    }
    G.raynorm = g->raynorm.empty() ? nullptr : g->d_raynorm.as<float4>();
    G.raytrap = g->raytrap.empty() ? nullptr : g->d_raytrap.as<float4>();
    G.kspan = g->kspan.empty() ? nullptr : g->d_kspan.as<float>();
    G.cov_off = nullptr;
    G.cov_idx = nullptr;
    set_bp3_bounds(G, d.sod, d.sdd, d.du, d.dv);
    G.fp_buf = (g->dim == 3 && (int64_t)d.nx * d.ny * ((d.nz + d.bz - 1) / d.bz) < ((int64_t)1 << 29)) ? 1 : 0;
    return upload_cover_index(g, st);
}

// ------------------------------------------------------------ projected-area weights

namespace {
struct P2 {
    double x, y;
};

double cross3(const P2& o, const P2& a, const P2& b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

// Convex hull (counter-clockwise, Andrew's monotone chain) of a few points.
std::vector<P2> hull(std::vector<P2> pts)
{
    std::sort(pts.begin(), pts.end(), [](const P2& a, const P2& b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
    std::vector<P2> h(2 * pts.size());
    size_t k = 0;
    for (size_t i = 0; i < pts.size(); ++i) {
        while (k >= 2 && cross3(h[k - 2], h[k - 1], pts[i]) <= 0) --k;
        h[k++] = pts[i];
    }
    for (size_t i = pts.size() - 1, t = k + 1; i-- > 0;) {
        while (k >= t && cross3(h[k - 2], h[k - 1], pts[i]) <= 0) --k;
        h[k++] = pts[i];
    }
    h.resize(k > 1 ? k - 1 : k);
    return h;
}

// Polygon clipped to the half-plane sgn * (coordinate axis) <= sgn * c (Sutherland-Hodgman).
std::vector<P2> clip(const std::vector<P2>& poly, int axis, double c, double sgn)
{
    std::vector<P2> out;
    const size_t n = poly.size();
    auto val = [&](const P2& p) { return sgn * ((axis == 0 ? p.x : p.y) - c); };
    for (size_t i = 0; i < n; ++i) {
        const P2& a = poly[i];
        const P2& b = poly[(i + 1) % n];
        const double va = val(a), vb = val(b);
        if (va <= 0) out.push_back(a);
        if ((va < 0 && vb > 0) || (va > 0 && vb < 0)) {
            const double t = va / (va - vb);
            out.push_back({a.x + t * (b.x - a.x), a.y + t * (b.y - a.y)});
        }
    }
    return out;
}

double area(const std::vector<P2>& poly)
{
    double a = 0.0;
    for (size_t i = 0; i < poly.size(); ++i) {
        const P2& p = poly[i];
        const P2& q = poly[(i + 1) % poly.size()];
        a += p.x * q.y - q.x * p.y;
    }
    return 0.5 * std::fabs(a);
}
}  // namespace

// im_area[v][s][j]: area, in detector pixels (pixel k spans [k - 1/2, k + 1/2]), of the
// part of column block j's projection in view v that falls on sub-detector s. The
// projection of a box is the convex hull of its corners' projections; in 2D the hull
// is an interval and the area its length. FP64.
static void projected_areas(bsgd_geometry* g)
{
    const bsgd_geometry_desc& d = g->d;
    const bool is3d = d.kind == BSGD_CONE_FLAT_3D, par = d.kind == BSGD_PARALLEL_2D;
    const double ku = 0.5 * (d.nu - 1), lv = 0.5 * (d.nv - 1);
    const double lox = -0.5 * d.nx * d.vx, loy = -0.5 * d.ny * d.vy, loz = -0.5 * d.nz * d.vz;
    g->im_area.assign((size_t)d.n_views * g->S * g->N, 0.0);
    for (int v = 0; v < d.n_views; ++v) {
        const double c = std::cos(d.angles_rad[v]), s = std::sin(d.angles_rad[v]);
        for (int j = 0; j < g->N; ++j) {
            const BlockInfo& B = g->blocks[j];
            std::vector<P2> pts;
            for (int q = 0; q < (is3d ? 8 : 4); ++q) {
                const double X = lox + ((q & 1) ? B.x0 + B.nbx : B.x0) * d.vx;
                const double Y = loy + ((q & 2) ? B.y0 + B.nby : B.y0) * d.vy;
                const double Z = loz + ((q & 4) ? B.z0 + B.nbz : B.z0) * d.vz;
                const double w = -X * s + Y * c;
                if (par) {
                    pts.push_back({w / d.du + ku, 0.0});
                } else {
                    const double dep = d.sod - (X * c + Y * s);
                    pts.push_back({d.sdd * w / dep / d.du + ku, is3d ? d.sdd * Z / dep / d.dv + lv : 0.0});
                }
            }
            if (!is3d) {
                double a = INFINITY, b = -INFINITY;
                for (const P2& p : pts) {
                    a = std::min(a, p.x);
                    b = std::max(b, p.x);
                }
                for (int sd = 0; sd < g->S; ++sd) {
                    const double s0 = (double)((sd * d.nu) / d.su) - 0.5, s1 = (double)(((sd + 1) * d.nu) / d.su) - 0.5;
                    g->im_area[((size_t)v * g->S + sd) * g->N + j] = std::max(0.0, std::min(b, s1) - std::max(a, s0));
                }
                continue;
            }
            const std::vector<P2> h = hull(pts);
            for (int sd = 0; sd < g->S; ++sd) {
                const int a = sd % d.su, b = sd / d.su;
                const double k0 = (double)((a * d.nu) / d.su) - 0.5, k1 = (double)(((a + 1) * d.nu) / d.su) - 0.5;
                const double l0 = (double)((b * d.nv) / d.sv) - 0.5, l1 = (double)(((b + 1) * d.nv) / d.sv) - 0.5;
                std::vector<P2> poly = clip(h, 0, k0, -1.0);
                poly = clip(poly, 0, k1, 1.0);
                poly = clip(poly, 1, l0, -1.0);
                poly = clip(poly, 1, l1, 1.0);
                g->im_area[((size_t)v * g->S + sd) * g->N + j] = poly.size() >= 3 ? area(poly) : 0.0;
            }
        }
    }
}

static bsgd_status compute_im(bsgd_geometry* g, hipStream_t st)
{
    const size_t n = (size_t)g->d.n_views * g->S * g->N;
    DevBuf dw, dn;
    g->bind(dw);
    g->bind(dn);
    HIP_TRY(dw.alloc(n * sizeof(double)));
    HIP_TRY(dn.alloc(n * sizeof(int64_t)));
    HIP_TRY(launch_geom_stats(g->dg, dw.as<double>(), dn.as<int64_t>(), st));
    g->im_w.resize(n);
    g->im_nnz.resize(n);
    HIP_TRY(hipMemcpyAsync(g->im_w.data(), dw.p, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(g->im_nnz.data(), dn.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    g->nnz_total = 0;
    for (int64_t c : g->im_nnz) g->nnz_total += c;

    g->im_q.assign(n, 0u);
    const bsgd_geometry_desc& d = g->d;
    if (d.im_table) {
        std::memcpy(g->im_q.data(), d.im_table, n * sizeof(uint32_t));
    } else if (d.im_mode == BSGD_IM_UNIFORM) {
        std::fill(g->im_q.begin(), g->im_q.end(), 1u);
    } else {
        // q = round(2^20 w / sum_s w), at least 1 where w > 0; w = the block column norm
        // (COLNORM) or the projected area (AREA)
        const std::vector<double>& W = d.im_mode == BSGD_IM_AREA ? g->im_area : g->im_w;
        for (int v = 0; v < d.n_views; ++v)
            for (int j = 0; j < g->N; ++j) {
                double tot = 0.0;
                for (int s = 0; s < g->S; ++s) tot += W[((size_t)v * g->S + s) * g->N + j];
                for (int s = 0; s < g->S; ++s) {
                    const size_t o = ((size_t)v * g->S + s) * g->N + j;
                    const double w = W[o];
                    uint32_t q = 0;
                    if (tot > 0.0) q = (uint32_t)std::floor(w / tot * (double)(1u << 20) + 0.5);
                    if (w > 0.0 && q == 0) q = 1;
                    g->im_q[o] = q;
                }
            }
    }
    HIP_TRY(g->d_q.alloc(n * sizeof(uint32_t)));
    HIP_TRY(hipMemcpyAsync(g->d_q.p, g->im_q.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_geometry_create(const bsgd_geometry_desc* desc, void* stream, bsgd_geometry** out)
{
    if (!out) return fail(BSGD_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    bsgd_status stt = validate(desc);
    if (stt != BSGD_OK) return stt;
    bsgd_geometry* g = new (std::nothrow) bsgd_geometry();
    if (!g) return fail(BSGD_E_OUT_OF_MEMORY, "host allocation failed");
    g->d = *desc;
    g->angles.assign(desc->angles_rad, desc->angles_rad + desc->n_views);
    g->d.angles_rad = g->angles.data();
    g->d.im_table = nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (desc->allocator) {
        g->alloc_copy = *desc->allocator;
        g->alloc = &g->alloc_copy;
    }
    g->d.allocator = g->alloc;
    g->st = st;
    g->bind_all();
    try {
        build_tables(g);
        projected_areas(g);
    } catch (...) {
        delete g;
        return fail(BSGD_E_OUT_OF_MEMORY, "host allocation failed while building tables");
    }
    stt = upload_tables(g, st);
    if (stt == BSGD_OK) {
        g->d.im_table = desc->im_table;
        stt = compute_im(g, st);
        g->d.im_table = nullptr;
    }
    if (stt != BSGD_OK) {
        delete g;
        return stt;
    }
    *out = g;
    return BSGD_OK;
}

extern "C" void bsgd_geometry_destroy(bsgd_geometry* g) { delete g; }

extern "C" bsgd_status bsgd_geometry_get_info(const bsgd_geometry* g, bsgd_geometry_info* out)
{
    if (!g || !out) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    out->n_rays = g->n_rays;
    out->n_voxels = g->n_vox;
    out->n_blocks = g->N;
    out->n_row_blocks = g->M;
    out->n_subdet = g->S;
    out->max_group_views = g->max_group;
    out->z_floats = g->z_floats;
    out->nnz = g->nnz_total;
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_geometry_table(const bsgd_geometry* g, int32_t which, void* out, size_t bytes)
{
    if (!g || !out) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    const void* src = nullptr;
    size_t need = 0;
    std::vector<int32_t> rects;
    switch (which) {
    case BSGD_TABLE_VIEW_ORDER:
        src = g->view_order.data();
        need = g->view_order.size() * sizeof(int32_t);
        break;
    case BSGD_TABLE_GROUP_START:
        src = g->group_start.data();
        need = g->group_start.size() * sizeof(int32_t);
        break;
    case BSGD_TABLE_IM_WEIGHTS:
        src = g->im_w.data();
        need = g->im_w.size() * sizeof(double);
        break;
    case BSGD_TABLE_IM_TABLE:
        src = g->im_q.data();
        need = g->im_q.size() * sizeof(uint32_t);
        break;
    case BSGD_TABLE_NNZ:
        src = g->im_nnz.data();
        need = g->im_nnz.size() * sizeof(int64_t);
        break;
    case BSGD_TABLE_IM_AREA:
        src = g->im_area.data();
        need = g->im_area.size() * sizeof(double);
        break;
    case BSGD_TABLE_FOOTPRINT:
        rects.resize(g->pairs.size() * 4);
        for (size_t i = 0; i < g->pairs.size(); ++i) {
            rects[4 * i] = g->pairs[i].u0;
            rects[4 * i + 1] = g->pairs[i].u1;
            rects[4 * i + 2] = g->pairs[i].v0;
            rects[4 * i + 3] = g->pairs[i].v1;
        }
        src = rects.data();
        need = rects.size() * sizeof(int32_t);
        break;
    default:
        return fail(BSGD_E_INVALID_ARG, "unknown table %d", which);
    }
    if (bytes < need) return fail(BSGD_E_INVALID_ARG, "table needs %zu bytes, got %zu", need, bytes);
    std::memcpy(out, src, need);
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_geometry_set_tuning(bsgd_geometry* g, const bsgd_tuning* t)
{
    if (!g || !t) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    if (t->fp_views_per_group < 1 || t->fp_views_per_group > FP_CHUNK_MAX)
        return fail(BSGD_E_INVALID_ARG, "fp_views_per_group must be in [1, %d]", FP_CHUNK_MAX);
    if (t->fp_ray_split != 1 && t->fp_ray_split != 2 && t->fp_ray_split != 4)
        return fail(BSGD_E_INVALID_ARG, "fp_ray_split must be 1, 2 or 4");
    if (t->fp_waves_per_pair < 0 || t->fp_waves_per_pair > 64)
        return fail(BSGD_E_INVALID_ARG, "fp_waves_per_pair must be in [1, 64] (0 keeps the current value)");
    if (t->bp_waves != 0 && t->bp_waves != 2 && t->bp_waves != 4 && t->bp_waves != 8)
        return fail(BSGD_E_INVALID_ARG, "bp_waves must be 2, 4 or 8 (0 keeps the current value)");
    for (int i = 0; i < 3; ++i)
        if (t->reserved[i] != 0) return fail(BSGD_E_INVALID_ARG, "reserved tuning fields must be 0");
    g->dg.fp_chunk = t->fp_views_per_group;
    g->dg.fp_split = t->fp_ray_split;
    if (t->fp_waves_per_pair > 0) g->dg.fp_wpp = t->fp_waves_per_pair;
    if (t->bp_waves > 0) g->dg.bp_split = t->bp_waves;
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_geometry_get_tuning(const bsgd_geometry* g, bsgd_tuning* t)
{
    if (!g || !t) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    std::memset(t, 0, sizeof *t);
    t->fp_views_per_group = g->dg.fp_chunk;
    t->fp_ray_split = g->dg.fp_split;
    t->fp_waves_per_pair = g->dg.fp_wpp;
    t->fp_staged = fp_lds_bytes_for(g->dg) > 0 ? 1 : 0;
    t->bp_waves = g->dg.bp_split;
    return BSGD_OK;
}

// Device view list for a standalone projector call.
static bsgd_status view_list(bsgd_geometry* g, const int32_t* views, int32_t n, hipStream_t st, const int32_t** dev)
{
    if (!views) {
        *dev = g->d_all_views.as<int32_t>();
        return BSGD_OK;
    }
    for (int i = 0; i < n; ++i)
        if (views[i] < 0 || views[i] >= g->d.n_views) return fail(BSGD_E_INVALID_ARG, "view index %d out of range", views[i]);
    const size_t b = (size_t)n * sizeof(int32_t);
    HIP_TRY(g->stage.reserve(b));
    std::memcpy(g->stage.host, views, b);
    if (g->d_views.bytes < b) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(g->d_views.alloc(std::max(b, (size_t)4096)));
    }
    HIP_TRY(g->stage.upload(g->d_views.p, b, st));
    *dev = g->d_views.as<int32_t>();
    return BSGD_OK;
}

// a: the image argument, b: the projections (NULL allowed when an empty view list selects none)
static bsgd_status check_proj_args(const bsgd_geometry* g, const void* a, const void* b, const int32_t* views,
                                   int32_t n_sel, int32_t block, uint32_t flags)
{
    if (!g || !a || (!b && !(views && n_sel == 0))) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    if (views && (n_sel < 0 || n_sel > 65535)) return fail(BSGD_E_INVALID_ARG, "n_views_sel must be in [0, 65535]");
    if (block < -1 || block >= g->N) return fail(BSGD_E_INVALID_ARG, "block %d out of range", block);
    if (flags & ~BSGD_ACCUMULATE) return fail(BSGD_E_INVALID_ARG, "unknown flags 0x%x", flags);
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_forward_project(const bsgd_geometry* gc, const float* x, float* y, const int32_t* views,
                                            int32_t n_sel, int32_t block, uint32_t flags, void* stream)
{
    bsgd_status stt = check_proj_args(gc, x, y, views, n_sel, block, flags);
    if (stt != BSGD_OK) return stt;
    bsgd_geometry* g = const_cast<bsgd_geometry*>(gc);
    hipStream_t st = (hipStream_t)stream;
    const int32_t* dv = nullptr;
    if (!views) n_sel = g->d.n_views;
    stt = view_list(g, views, n_sel, st, &dv);
    if (stt != BSGD_OK) return stt;
    HIP_TRY(launch_fp_full(g->dg, dv, n_sel, block, x, y, (flags & BSGD_ACCUMULATE) ? 1 : 0, st));
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_back_project(const bsgd_geometry* gc, const float* y, float* x, const int32_t* views,
                                         int32_t n_sel, int32_t block, float scale, uint32_t flags, void* stream)
{
    bsgd_status stt = check_proj_args(gc, x, y, views, n_sel, block, flags);
    if (stt != BSGD_OK) return stt;
    if (!std::isfinite(scale)) return fail(BSGD_E_INVALID_ARG, "scale must be finite");
    bsgd_geometry* g = const_cast<bsgd_geometry*>(gc);
    hipStream_t st = (hipStream_t)stream;
    const int32_t* dv = nullptr;
    if (!views) n_sel = g->d.n_views;
    stt = view_list(g, views, n_sel, st, &dv);
    if (stt != BSGD_OK) return stt;
    HIP_TRY(launch_bp_full(g->dg, dv, n_sel, block, y, x, scale, (flags & BSGD_ACCUMULATE) ? 1 : 0, st));
    return BSGD_OK;
}

// ------------------------------------------------------------ solver

enum { KID_FP = 0, KID_RESID = 1, KID_BP = 2, KID_TV = 3, KID_DRAW = 4, KID_COUNT = 5 };

static void drop_batch_graphs(const bsgd_solver* s);

struct bsgd_solver {
    const bsgd_geometry* g = nullptr;
    const float* y = nullptr;
    float* x = nullptr;
    bsgd_options o{};
    hipStream_t st = nullptr;
    int R = 1, B = 1, T = 1, tv_every = 1, maxv = 1;
    int64_t k = 0;
    bool failed = false, im = false, subdet = false;
    SchedLayout L{};
    DevBuf z, ghat, gsum, r_sel, sched, draws, work, partials, norm_out, tv_p, tv_a, tv_b;
    DevBuf rho, delta;  // sub-detector memory: residual snapshots and their changes (z layout)
    // global-memory forward walk: x stored y fastest ([z][x][y]), refreshed from x at the
    // start of every step call and after every TV prox, and written with x by the back
    // projection in between; unallocated otherwise
    DevBuf xT;
    int sched_cap = 0;
    Staging stage;
    // one captured epoch (T iterations) replayed per epoch
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    DevBuf g_sched, g_work, g_draws;
    // entry table of batched calls led by this solver
    // step length on the device (read by the back-projection kernel) and Algorithm 3
    DevBuf mu_dev, eud_cur, eud_prev;
    DevBuf tv_w;             // {w = mu lambda, dual step} of the TV prox, on the device
    float* tv_w_host = nullptr;
    DevBuf nr_ty, nr_tg;   // normal-residual scratch (bsgd_normal_residual)
    DevBuf nr_out;         // {||A^T (y - A x)||^2, ||A^T y||^2} of the last asynchronous check
    bool nr_ref_dev = false;  // nr_out[1] holds ||A^T y||^2
    double nr_ref = -1.0;  // ||A^T y||, once computed
    float* mu_host = nullptr;
    double mu_cur = 0.0;
    bool auto_mu = false, have_prev_eud = false;
    double prev_eud_n2 = 0.0;
    double am_eps = 0.05, am_delta = 0.4, am_t1 = 0.1, am_t2 = 0.5;
    std::vector<double> r_hist, theta_hist, mu_hist;
    double* norm_host = nullptr;
    // last call's schedule (host) for export
    std::vector<int32_t> last_sched;
    int last_n = 0;
    // profiling
    bool prof = false;
    hipEvent_t last_use = nullptr;  // recorded after each call's work on the stream
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double ms[KID_COUNT] = {0, 0, 0, 0, 0};
    int64_t launches[KID_COUNT] = {0, 0, 0, 0, 0};

    ~bsgd_solver()
    {
        // With an allocator the device buffers return to it in stream order; then only
        // this solver's own work has to finish (its last-use event), not the stream.
        if (last_use && g && g->alloc)
            (void)hipEventSynchronize(last_use);
        else if (st)
            (void)hipStreamSynchronize(st);
        if (last_use) (void)hipEventDestroy(last_use);
        drop_batch_graphs(this);
        for (auto& p : pending) {
            ev_pool.push_back(p.second.first);
            ev_pool.push_back(p.second.second);
        }
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        pinned_put(norm_host, 4 * sizeof(double));
        pinned_put(mu_host, sizeof(float));
        pinned_put(tv_w_host, 2 * sizeof(float));
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    hipError_t event(hipEvent_t* e)
    {
        if (!ev_pool.empty()) {
            *e = ev_pool.back();
            ev_pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
};

// Launch helper recording a start/stop event pair around `fn` when profiling.
template <class F>
static hipError_t timed(bsgd_solver* s, int kid, F&& fn)
{
    if (!s->prof) return fn();
    hipEvent_t a, b;
    hipError_t e = s->event(&a);
    if (e != hipSuccess) return e;
    e = s->event(&b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a, s->st);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s->st);
    if (e != hipSuccess) return e;
    s->pending.push_back({kid, {a, b}});
    s->launches[kid] += 1;
    return hipSuccess;
}

// Record that the solver's work so far has been enqueued on st (its destructor waits for
// this point instead of the whole stream when the memory is stream-ordered).
static void mark_use(const bsgd_solver* s, hipStream_t st)
{
    if (s->last_use) (void)hipEventRecord(s->last_use, st);
}

static bsgd_status resolve_counts(const bsgd_geometry* g, const bsgd_options* o, int& R, int& B)
{
    if (o->rows_per_iter == 0 && o->blocks_per_iter == 0) {
        const int P = o->node_count;
        if (P < 1) return fail(BSGD_E_INVALID_ARG, "give rows_per_iter and blocks_per_iter, or node_count >= 1");
        B = std::min(P, g->N);  // gamma N = min(N, P)
        if (P % B) return fail(BSGD_E_INVALID_ARG, "node_count %d gives a non-integer alpha M", P);
        R = P / B;  // alpha M = P / (N gamma)
        if (R > g->M) return fail(BSGD_E_INVALID_ARG, "node_count %d exceeds M N", P);
        return BSGD_OK;
    }
    R = o->rows_per_iter;
    B = o->blocks_per_iter;
    if (R < 1 || R > g->M) return fail(BSGD_E_INVALID_ARG, "rows_per_iter must be in [1, M]");
    if (B < 1 || B > g->N) return fail(BSGD_E_INVALID_ARG, "blocks_per_iter must be in [1, N]");
    return BSGD_OK;
}

static bsgd_status solver_create(const bsgd_geometry* g, const float* y, float* x, const bsgd_options* o,
                                 hipStream_t st, bsgd_solver** out)
{
    if (!g || !y || !x || !o || !out) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    int R, B;
    bsgd_status stt = resolve_counts(g, o, R, B);
    if (stt != BSGD_OK) return stt;
    if (!std::isfinite(o->mu)) return fail(BSGD_E_INVALID_ARG, "mu must be finite");
    if (!(o->tv_lambda >= 0.0) || !std::isfinite(o->tv_lambda)) return fail(BSGD_E_INVALID_ARG, "tv_lambda must be >= 0");
    if (o->tv_lambda > 0 && o->tv_inner_iters < 1) return fail(BSGD_E_INVALID_ARG, "tv_inner_iters must be >= 1");
    if (o->tv_every < 0 || o->max_effective_epochs < 0 || o->check_every < 0 || !(o->tol >= 0.0))
        return fail(BSGD_E_INVALID_ARG, "negative option");
    if (o->im_until < 0) return fail(BSGD_E_INVALID_ARG, "im_until must be >= 0");
    if (o->flags & ~(BSGD_FLAG_EAGER | BSGD_FLAG_SUBDET_MEMORY)) return fail(BSGD_E_INVALID_ARG, "unknown flag");
    if (o->auto_mu && (!(o->mu_eps >= 0) || !(o->mu_delta >= 0 && o->mu_delta < 1) || !(o->mu_t1 >= 0) ||
                       !(o->mu_t2 >= 0) || !(o->mu > 0)))
        return fail(BSGD_E_INVALID_ARG, "auto_mu needs mu > 0, eps >= 0, 0 <= delta < 1, t1, t2 >= 0");
    bsgd_solver* s = new (std::nothrow) bsgd_solver();
    if (!s) return fail(BSGD_E_OUT_OF_MEMORY, "host allocation failed");
    s->g = g;
    s->y = y;
    s->x = x;
    s->o = *o;
    s->st = st;
    s->R = R;
    s->B = B;
    s->T = std::max(1, (int)std::lround((double)g->M * g->N / ((double)R * B)));
    s->tv_every = o->tv_every > 0 ? o->tv_every : s->T;
    s->maxv = R * g->max_group;
    s->im = g->d.im_mode != BSGD_IM_NONE;
    s->L.R = R;
    s->L.B = B;
    s->L.maxv = s->maxv;
    s->L.stride = SchedLayout::stride_for(R, B, s->maxv);
    s->graphs = (o->flags & BSGD_FLAG_EAGER) == 0;
    s->subdet = (o->flags & BSGD_FLAG_SUBDET_MEMORY) != 0;
    for (DevBuf* b : {&s->z, &s->ghat, &s->gsum, &s->r_sel, &s->sched, &s->draws, &s->work, &s->partials, &s->norm_out,
                      &s->tv_p, &s->tv_a, &s->tv_b, &s->rho, &s->delta, &s->g_sched, &s->g_work, &s->g_draws,
                      &s->mu_dev, &s->eud_cur, &s->eud_prev, &s->tv_w, &s->nr_ty, &s->nr_tg, &s->nr_out, &s->xT})
        b->use(g->alloc, st);
    const int64_t per_view = (int64_t)g->d.nu * g->d.nv;
    auto cleanup = [&](bsgd_status e) {
        delete s;
        return e;
    };
#define S_TRY(expr)                                                                                \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return cleanup(fail(e_ == hipErrorOutOfMemory ? BSGD_E_OUT_OF_MEMORY : BSGD_E_DEVICE, "%s: %s", #expr, \
                                hipGetErrorString(e_)));                                           \
    } while (0)
    S_TRY(s->z.alloc((size_t)g->z_floats * sizeof(float)));
    if (s->subdet) {
        S_TRY(s->rho.alloc((size_t)g->z_floats * sizeof(float)));
        S_TRY(s->delta.alloc((size_t)g->z_floats * sizeof(float)));
    } else {
        S_TRY(s->ghat.alloc((size_t)g->M * g->n_vox * sizeof(float)));
    }
    S_TRY(s->gsum.alloc((size_t)g->n_vox * sizeof(float)));
    if (fp_lds_bytes_for(g->dg) == 0) S_TRY(s->xT.alloc((size_t)g->n_vox * sizeof(float)));
    // 2D: one {w2, slope, lmax, r} record per selected ray; 3D: the residual
    S_TRY(s->r_sel.alloc((size_t)s->maxv * per_view * (g->dim == 2 ? 4 : 1) * sizeof(float)));
    const int n_part = (int)(((per_view + 255) / 256) * g->d.n_views);
    S_TRY(s->partials.alloc((size_t)std::max(n_part, 4096) * sizeof(double)));
    S_TRY(s->norm_out.alloc(4 * sizeof(double)));
    S_TRY(pinned_get((void**)&s->norm_host, 4 * sizeof(double), nullptr));
    S_TRY(s->mu_dev.alloc(sizeof(float)));
    S_TRY(pinned_get((void**)&s->mu_host, sizeof(float), nullptr));
    s->mu_cur = o->mu;
    *s->mu_host = (float)o->mu;
    S_TRY(hipMemcpyAsync(s->mu_dev.p, s->mu_host, sizeof(float), hipMemcpyHostToDevice, st));
    S_TRY(hipStreamSynchronize(st));
    s->auto_mu = o->auto_mu != 0;
    if (s->auto_mu) {
        if (o->mu_eps > 0) s->am_eps = o->mu_eps;
        if (o->mu_delta > 0) s->am_delta = o->mu_delta;
        if (o->mu_t1 > 0) s->am_t1 = o->mu_t1;
        if (o->mu_t2 > 0) s->am_t2 = o->mu_t2;
        S_TRY(s->eud_cur.alloc((size_t)g->n_vox * sizeof(float)));
        S_TRY(s->eud_prev.alloc((size_t)g->n_vox * sizeof(float)));
        S_TRY(launch_fill(s->eud_cur.as<float>(), 0.0f, g->n_vox, st));
    }
    if (o->tv_lambda > 0) {
        const size_t nb = (size_t)g->dim * g->n_vox * sizeof(float);
        S_TRY(s->tv_p.alloc(nb));  // three dual iterates in rotation
        S_TRY(s->tv_a.alloc(nb));
        S_TRY(s->tv_b.alloc(nb));
        S_TRY(s->tv_w.alloc(2 * sizeof(float)));
        S_TRY(pinned_get((void**)&s->tv_w_host, 2 * sizeof(float), nullptr));
        tv_weight_step(g->dim, o->mu, o->tv_lambda, s->tv_w_host);
        S_TRY(hipMemcpyAsync(s->tv_w.p, s->tv_w_host, 2 * sizeof(float), hipMemcpyHostToDevice, st));
        S_TRY(hipStreamSynchronize(st));
    }
    S_TRY(launch_fill(s->z.as<float>(), 0.0f, g->z_floats, st));
    if (s->subdet)
        S_TRY(launch_fill(s->rho.as<float>(), 0.0f, g->z_floats, st));
    else
        S_TRY(launch_fill(s->ghat.as<float>(), 0.0f, (int64_t)g->M * g->n_vox, st));
    S_TRY(launch_fill(s->gsum.as<float>(), 0.0f, g->n_vox, st));
    S_TRY(hipEventCreateWithFlags(&s->last_use, hipEventDisableTiming));
    mark_use(s, st);
#undef S_TRY
    *out = s;
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_create(const bsgd_geometry* g, const float* y, float* x, const bsgd_options* o,
                                          void* stream, bsgd_solver** out)
{
    return solver_create(g, y, x, o, (hipStream_t)stream, out);
}

extern "C" void bsgd_solver_destroy(bsgd_solver* s) { delete s; }

static bsgd_status ensure_sched(bsgd_solver* s, int n)
{
    if (n <= s->sched_cap) return BSGD_OK;
    HIP_TRY(hipStreamSynchronize(s->st));
    const int cap = std::max(n, 64);
    HIP_TRY(s->sched.alloc((size_t)cap * s->L.stride * sizeof(int32_t)));
    HIP_TRY(s->work.alloc((size_t)cap * s->maxv * s->B * sizeof(PairWork)));
    if (s->im) HIP_TRY(s->draws.alloc((size_t)cap * s->maxv * s->B));
    s->sched_cap = cap;
    return BSGD_OK;
}

static void fill_schedule(bsgd_solver* s, int n, int32_t* out)
{
    const bsgd_geometry* g = s->g;
    const SchedLayout& L = s->L;
    std::vector<int32_t> scratch;
    for (int it = 0; it < n; ++it) {
        int32_t* rec = out + (size_t)it * L.stride;
        std::fill(rec, rec + L.stride, 0);
        const int64_t k = s->k + it;
        choose(s->o.seed, STREAM_ROWS, k, g->M, L.R, rec + L.off_rows(), scratch);
        choose(s->o.seed, STREAM_BLOCKS, k, g->N, L.B, rec + L.off_blocks(), scratch);
        int nv = 0;
        for (int ri = 0; ri < L.R; ++ri) {
            const int i = rec[L.off_rows() + ri];
            rec[L.off_gstart() + ri] = nv;
            for (int p = g->group_start[i]; p < g->group_start[i + 1]; ++p) rec[L.off_views() + nv++] = g->view_order[p];
        }
        rec[L.off_gstart() + L.R] = nv;
        rec[0] = nv;
        rec[L.off_k()] = (int32_t)(uint32_t)((uint64_t)k & 0xffffffffu);
        rec[L.off_k() + 1] = (int32_t)(uint32_t)((uint64_t)k >> 32);
    }
}

static bsgd_status resid_norm(bsgd_solver* s, double* out)
{
    int np = 0;
    HIP_TRY(launch_resid_sumsq(s->g->dg, s->y, s->z.as<float>(), s->partials.as<double>(), &np, s->st));
    HIP_TRY(launch_sum_partials(s->partials.as<double>(), np, s->norm_out.as<double>(), s->st));
    HIP_TRY(hipMemcpyAsync(s->norm_host, s->norm_out.p, sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    *out = std::sqrt(*s->norm_host);
    return BSGD_OK;
}

// Enqueue n_iters iterations reading schedule records `dsched` and writing work
// records / draws into `dwork` / `ddraws`; k_first is the counter of the first one
// (used only to place the TV steps).
// The copy of x stored y fastest, from x (no-op when the solver keeps none).
static hipError_t refresh_xT(bsgd_solver* s, hipStream_t st)
{
    if (!s->xT.p) return hipSuccess;
    const bsgd_geometry_desc& d = s->g->d;
    return launch_xy_transpose(s->x, s->xT.as<float>(), d.nx, d.ny, d.nz, st);
}

static hipError_t enqueue_iterations(bsgd_solver* s, hipStream_t st, const int32_t* dsched, PairWork* dwork,
                                     int8_t* ddraws, int n_iters, int64_t k_first)
{
    const bsgd_geometry* g = s->g;
    hipError_t e = timed(s, KID_DRAW, [&] {
        return launch_plan(g->dg, dsched, s->L, n_iters, s->o.seed, s->im ? g->d_q.as<uint32_t>() : nullptr,
                           (int64_t)s->o.im_until, ddraws,
                           dwork, st);
    });
    if (e != hipSuccess) return e;
    const int64_t per_it_work = (int64_t)s->maxv * s->B;
    for (int it = 0; it < n_iters; ++it) {
        const int32_t* rec = dsched + (size_t)it * s->L.stride;
        const PairWork* wk = dwork + it * per_it_work;
        e = timed(s, KID_FP, [&] {
            return launch_fp_pairs(g->dg, wk, s->L, rec + s->L.off_blocks(), s->x, s->xT.as<float>(), s->z.as<float>(),
                                   st);
        });
        if (e != hipSuccess) return e;
        e = timed(s, KID_RESID, [&] {
            hipError_t e2 = launch_resid(g->dg, rec, s->L, s->y, s->z.as<float>(), s->r_sel.as<float>(), st);
            if (e2 == hipSuccess && s->subdet)
                e2 = launch_subdet_delta(g->dg, rec, wk, s->L, s->r_sel.as<float>(), s->rho.as<float>(),
                                         s->delta.as<float>(), st);
            return e2;
        });
        if (e != hipSuccess) return e;
        e = timed(s, KID_BP, [&] {
            return launch_bp_step(g->dg, rec, wk, s->L, s->r_sel.as<float>(), s->subdet ? s->delta.as<float>() : nullptr,
                                  s->ghat.as<float>(), s->gsum.as<float>(), s->x, s->xT.as<float>(), s->mu_dev.as<float>(),
                                  g->n_vox, st);
        });
        if (e != hipSuccess) return e;
        if (s->auto_mu) {
            e = launch_add(s->eud_cur.as<float>(), s->gsum.as<float>(), g->n_vox, st);
            if (e != hipSuccess) return e;
        }
        // the prox reads its weight mu lambda from the device (Algorithm 3 may change mu
        // between replays of a captured epoch); a non-positive weight is the identity
        if (s->o.tv_lambda > 0 && (s->auto_mu || s->mu_cur > 0) && (k_first + it + 1) % s->tv_every == 0) {
            e = timed(s, KID_TV, [&] {
                hipError_t e2 = launch_tv_prox(g->dg, s->x, s->tv_w.as<float>(), s->o.tv_inner_iters,
                                               s->tv_p.as<float>(), s->tv_a.as<float>(), s->tv_b.as<float>(), st);
                return e2 == hipSuccess ? refresh_xT(s, st) : e2;
            });
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Capture one epoch (T iterations starting at a multiple of T) on a private stream.
static bsgd_status build_graph(bsgd_solver* s)
{
    const int T = s->T;
    HIP_TRY(s->g_sched.alloc((size_t)T * s->L.stride * sizeof(int32_t)));
    HIP_TRY(s->g_work.alloc((size_t)T * s->maxv * s->B * sizeof(PairWork)));
    if (s->im) HIP_TRY(s->g_draws.alloc((size_t)T * s->maxv * s->B));
    HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_iterations(s, s->cap_stream, s->g_sched.as<int32_t>(), s->g_work.as<PairWork>(),
                                      s->im ? s->g_draws.as<int8_t>() : nullptr, T, 0);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(BSGD_E_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    s->graph = graph;
    HIP_TRY(hipGraphInstantiate(&s->graph_exec, graph, nullptr, nullptr, 0));
    return BSGD_OK;
}

static bsgd_status step_segment(bsgd_solver* s, int n_iters)
{
    const int T = s->T;
    const bool tv_aligned = !(s->o.tv_lambda > 0) || (T % s->tv_every == 0);
    const bool use_graph =
        s->graphs && !s->prof && n_iters % T == 0 && s->k % T == 0 && tv_aligned && n_iters > 0;
    bsgd_status stt = ensure_sched(s, n_iters);
    if (stt != BSGD_OK) return stt;
    HIP_TRY(refresh_xT(s, s->st));  // the caller may have changed x since the last call
    const size_t sched_bytes = (size_t)n_iters * s->L.stride * sizeof(int32_t);
    HIP_TRY(s->stage.reserve(sched_bytes));
    int32_t* host = reinterpret_cast<int32_t*>(s->stage.host);
    fill_schedule(s, n_iters, host);
    s->last_sched.assign(host, host + (size_t)n_iters * s->L.stride);
    s->last_n = n_iters;
    if (!use_graph) {
        HIP_TRY(s->stage.upload(s->sched.p, sched_bytes, s->st));
        HIP_TRY(enqueue_iterations(s, s->st, s->sched.as<int32_t>(), s->work.as<PairWork>(),
                                   s->im ? s->draws.as<int8_t>() : nullptr, n_iters, s->k));
        s->k += n_iters;
        return BSGD_OK;
    }
    if (!s->graph_exec) {
        stt = build_graph(s);
        if (stt != BSGD_OK) return stt;
    }
    const size_t epoch_sched = (size_t)T * s->L.stride * sizeof(int32_t);
    const size_t epoch_draws = (size_t)T * s->maxv * s->B;
    for (int e = 0; e < n_iters / T; ++e) {
        HIP_TRY(hipMemcpyAsync(s->g_sched.p, reinterpret_cast<char*>(s->stage.host) + e * epoch_sched, epoch_sched,
                               hipMemcpyHostToDevice, s->st));
        HIP_TRY(hipGraphLaunch(s->graph_exec, s->st));
        if (s->im)
            HIP_TRY(hipMemcpyAsync(s->draws.as<int8_t>() + e * epoch_draws, s->g_draws.p, epoch_draws,
                                   hipMemcpyDeviceToDevice, s->st));
    }
    HIP_TRY(hipEventRecord(s->stage.done, s->st));
    s->stage.pending = true;
    s->k += n_iters;
    return BSGD_OK;
}

// Algorithm 3 check at an iteration count that is a multiple of M: EUD norms, the
// cosine between consecutive EUDs, the residual norm, then the two criteria.
static bsgd_status auto_mu_check(bsgd_solver* s)
{
    const bsgd_geometry* g = s->g;
    double* dp = s->partials.as<double>();
    double* out = s->norm_out.as<double>();
    int np = 0;
    HIP_TRY(launch_dot(s->eud_cur.as<float>(), s->eud_cur.as<float>(), g->n_vox, dp, &np, s->st));
    HIP_TRY(launch_sum_partials(dp, np, out, s->st));
    if (s->have_prev_eud) {
        HIP_TRY(launch_dot(s->eud_cur.as<float>(), s->eud_prev.as<float>(), g->n_vox, dp, &np, s->st));
        HIP_TRY(launch_sum_partials(dp, np, out + 1, s->st));
    }
    HIP_TRY(launch_resid_sumsq(g->dg, s->y, s->z.as<float>(), dp, &np, s->st));
    HIP_TRY(launch_sum_partials(dp, np, out + 2, s->st));
    HIP_TRY(hipMemcpyAsync(s->norm_host, out, 3 * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    const double n2 = s->norm_host[0], cross = s->norm_host[1], r = std::sqrt(s->norm_host[2]);
    s->r_hist.push_back(r);
    if (s->have_prev_eud) s->theta_hist.push_back(cross / std::sqrt(n2 * s->prev_eud_n2));
    const size_t nr = s->r_hist.size(), nt = s->theta_hist.size();
    if (nr >= 3 && nt >= 2) {
        const double r0 = s->r_hist[nr - 1], r1 = s->r_hist[nr - 2], r2 = s->r_hist[nr - 3];
        const double th = s->theta_hist[nt - 1], thp = s->theta_hist[nt - 2];
        double mu = s->mu_cur;
        if (r0 < r1 && r1 < r2) mu = (1.0 + s->am_eps) * mu;
        if (r0 > r1 && r1 > r2 && (std::fabs(th - thp) > s->am_t1 || th < s->am_t2)) mu = (1.0 - s->am_delta) * mu;
        if (mu != s->mu_cur) {
            s->mu_cur = mu;
            *s->mu_host = (float)mu;
            HIP_TRY(hipMemcpyAsync(s->mu_dev.p, s->mu_host, sizeof(float), hipMemcpyHostToDevice, s->st));
            if (s->tv_w_host) {
                tv_weight_step(g->dim, mu, s->o.tv_lambda, s->tv_w_host);
                HIP_TRY(hipMemcpyAsync(s->tv_w.p, s->tv_w_host, 2 * sizeof(float), hipMemcpyHostToDevice, s->st));
            }
            HIP_TRY(hipStreamSynchronize(s->st));
        }
    }
    s->mu_hist.push_back(s->mu_cur);
    s->prev_eud_n2 = n2;
    s->have_prev_eud = true;
    HIP_TRY(hipMemcpyAsync(s->eud_prev.p, s->eud_cur.p, (size_t)g->n_vox * sizeof(float), hipMemcpyDeviceToDevice,
                           s->st));
    HIP_TRY(launch_fill(s->eud_cur.as<float>(), 0.0f, g->n_vox, s->st));
    return BSGD_OK;
}

static bsgd_status step_impl(bsgd_solver* s, int n_iters)
{
    if (!s->auto_mu) return step_segment(s, n_iters);
    const int M = s->g->M;
    int left = n_iters;
    while (left > 0) {
        const int seg = std::min<int64_t>(left, M - s->k % M);
        bsgd_status stt = step_segment(s, seg);
        if (stt != BSGD_OK) return stt;
        left -= seg;
        if (s->k % M == 0) {
            stt = auto_mu_check(s);
            if (stt != BSGD_OK) return stt;
        }
    }
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_step_length(const bsgd_solver* s, double* mu_now, double* history, int32_t cap,
                                              int32_t* n_history)
{
    if (!s) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    if (mu_now) *mu_now = s->mu_cur;
    if (n_history) *n_history = (int32_t)s->mu_hist.size();
    if (history)
        for (int32_t i = 0; i < cap && i < (int32_t)s->mu_hist.size(); ++i) history[i] = s->mu_hist[i];
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_step(bsgd_solver* s, int32_t n_iters, double* resid_norm_out)
{
    if (!s) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    if (s->failed) return fail(BSGD_E_STATE, "solver is in a failed state");
    if (n_iters < 0 || n_iters > (1 << 20)) return fail(BSGD_E_INVALID_ARG, "n_iters must be in [0, 2^20]");
    if (n_iters > 0) {
        bsgd_status stt = step_impl(s, n_iters);
        if (stt != BSGD_OK) {
            s->failed = true;
            return stt;
        }
    }
    mark_use(s, s->st);
    if (resid_norm_out) {
        bsgd_status stt = resid_norm(s, resid_norm_out);
        if (stt != BSGD_OK) {
            s->failed = true;
            return stt;
        }
        if (!std::isfinite(*resid_norm_out)) return fail(BSGD_E_DIVERGED, "residual norm is not finite");
    }
    return BSGD_OK;
}

// Schedule and upload n_iters iterations of one solver on stream st (no kernels).
static bsgd_status upload_iterations(bsgd_solver* s, int n_iters, hipStream_t st)
{
    bsgd_status stt = ensure_sched(s, n_iters);
    if (stt != BSGD_OK) return stt;
    const size_t sched_bytes = (size_t)n_iters * s->L.stride * sizeof(int32_t);
    HIP_TRY(s->stage.reserve(sched_bytes));
    int32_t* host = reinterpret_cast<int32_t*>(s->stage.host);
    fill_schedule(s, n_iters, host);
    s->last_sched.assign(host, host + (size_t)n_iters * s->L.stride);
    s->last_n = n_iters;
    HIP_TRY(s->stage.upload(s->sched.p, sched_bytes, st));
    return BSGD_OK;
}

// The plan (draws and work records) of n_iters uploaded iterations.
static hipError_t plan_iterations(bsgd_solver* s, int n_iters, hipStream_t st)
{
    const bsgd_geometry* g = s->g;
    return launch_plan(g->dg, s->sched.as<int32_t>(), s->L, n_iters, s->o.seed,
                       s->im ? g->d_q.as<uint32_t>() : nullptr, (int64_t)s->o.im_until,
                       s->im ? s->draws.as<int8_t>() : nullptr, s->work.as<PairWork>(), st);
}

// Launch groups of a batched call: up to BATCH_GROUP entries each (passed as kernel
// arguments), the LDS-staged forward projections first, sorted by LDS size (the order
// of the entries does not affect any solve's arithmetic).
struct BatchLaunchGroup {
    BatchArgs A;
    int wgs[3];
    std::vector<FpLaunchClass> classes;
    std::vector<BpLaunchClass> bp_classes;
    size_t res_lds;
};

static std::vector<BatchLaunchGroup> batch_groups(bsgd_solver* const* solvers, int n)
{
    std::vector<bsgd_solver*> order(solvers, solvers + n);
    // forward-projection LDS size descending, then the 2D back projection's wave split, so
    // each launch class is one contiguous run of workgroups
    std::stable_sort(order.begin(), order.end(), [](const bsgd_solver* a, const bsgd_solver* b) {
        const size_t la = fp_lds_bytes_for(a->g->dg), lb = fp_lds_bytes_for(b->g->dg);
        if (la != lb) return la > lb;
        return a->g->dg.bp_split < b->g->dg.bp_split;
    });
    std::vector<BatchLaunchGroup> groups;
    for (int g0 = 0; g0 < n; g0 += BATCH_GROUP) {
        groups.emplace_back();
        BatchLaunchGroup& grp = groups.back();
        std::memset(&grp.A, 0, sizeof grp.A);
        grp.wgs[0] = grp.wgs[1] = grp.wgs[2] = 0;
        grp.res_lds = 0;
        const int m = std::min(BATCH_GROUP, n - g0);
        for (int i = 0; i < m; ++i) {
            bsgd_solver* s = order[g0 + i];
            BatchEntry& e = grp.A.e[i];
            e.G = s->g->dg;
            e.L = s->L;
            e.sched = s->sched.as<int32_t>();
            e.work = s->work.as<PairWork>();
            e.y = s->y;
            e.x = s->x;
            e.xT = s->xT.as<float>();
            e.z = s->z.as<float>();
            e.ghat = s->ghat.as<float>();
            e.gsum = s->gsum.as<float>();
            e.r_sel = s->r_sel.as<float>();
            e.mu = s->mu_dev.as<float>();
            e.n_vox = s->g->n_vox;
            batch_grids(e);
            const int per[3] = {e.gx[0] * (e.fp_lds ? e.L.B : 1), e.gx[1] * e.L.maxv, e.gx[2] * e.L.B};
            for (int p = 0; p < 3; ++p) {
                e.base[p] = grp.wgs[p];
                grp.wgs[p] += per[p];
            }
            const size_t lb = e.fp_lds ? fp_lds_bytes_for(e.G) : (size_t)0;
            if (grp.classes.empty() || grp.classes.back().lds_bytes != lb)
                grp.classes.push_back({(int)e.base[0], 0, lb});
            grp.classes.back().wgs += per[0];
            if (grp.bp_classes.empty() || grp.bp_classes.back().split != e.G.bp_split)
                grp.bp_classes.push_back({(int)e.base[2], 0, (int)e.G.bp_split});
            grp.bp_classes.back().wgs += per[2];
            grp.res_lds = std::max(grp.res_lds, resid_lds_bytes_for(e.G));
        }
        grp.A.n = m;
    }
    return groups;
}

// The iterations of a batched call (after their plans): per iteration one launch per
// phase and group, then the TV steps due (k0 = the solvers' common counter before the
// call when `aligned`, else each solver's own).
static hipError_t enqueue_batch(std::vector<BatchLaunchGroup>& groups, bsgd_solver* const* solvers, int n,
                                int n_iters, int dim, hipStream_t st)
{
    for (int it = 0; it < n_iters; ++it) {
        for (BatchLaunchGroup& grp : groups) {
            grp.A.it = it;
            hipError_t he = launch_batch_iteration(grp.A, dim, grp.wgs, grp.classes.data(), (int)grp.classes.size(),
                                                   grp.bp_classes.data(), (int)grp.bp_classes.size(), grp.res_lds, st);
            if (he != hipSuccess) return he;
        }
        for (int i = 0; i < n; ++i) {
            bsgd_solver* s = solvers[i];
            if (s->o.tv_lambda > 0 && s->mu_cur > 0 && (s->k + it + 1) % s->tv_every == 0) {
                hipError_t he = launch_tv_prox(s->g->dg, s->x, s->tv_w.as<float>(), s->o.tv_inner_iters,
                                               s->tv_p.as<float>(), s->tv_a.as<float>(), s->tv_b.as<float>(), st);
                if (he == hipSuccess) he = refresh_xT(s, st);
                if (he != hipSuccess) return he;
            }
        }
    }
    return hipSuccess;
}

// Captured batched epochs: one graph per ordered set of solvers (one effective epoch from
// an epoch boundary, plans included), replayed while the set recurs. A set is captured
// the second time in a row it is stepped; a few graphs are kept, and a solver's
// destruction drops the graphs that hold it.
namespace {
struct BatchGraph {
    std::vector<bsgd_solver*> key;
    std::vector<const void*> bufs;  // buffers baked into the graph, per solver: sched, work, draws
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};
constexpr size_t BATCH_GRAPHS_KEPT = 16;
std::mutex g_bg_mu;
std::vector<std::unique_ptr<BatchGraph>> g_bg;  // most recently used last
std::vector<bsgd_solver*> g_bg_last;            // the set of the previous graph-eligible call
}  // namespace

static std::vector<const void*> batch_bufs(bsgd_solver* const* solvers, int n)
{
    std::vector<const void*> b;
    for (int i = 0; i < n; ++i) {
        b.push_back(solvers[i]->sched.p);
        b.push_back(solvers[i]->work.p);
        b.push_back(solvers[i]->draws.p);
    }
    return b;
}

static void drop_batch_graphs(const bsgd_solver* s)
{
    std::lock_guard<std::mutex> lock(g_bg_mu);
    for (size_t i = 0; i < g_bg.size();) {
        if (std::find(g_bg[i]->key.begin(), g_bg[i]->key.end(), s) != g_bg[i]->key.end())
            g_bg.erase(g_bg.begin() + i);
        else
            ++i;
    }
    if (std::find(g_bg_last.begin(), g_bg_last.end(), s) != g_bg_last.end()) g_bg_last.clear();
}

static bsgd_status capture_batch_graph(bsgd_solver* const* solvers, int n, int dim, std::unique_ptr<BatchGraph>& out)
{
    auto bg = std::make_unique<BatchGraph>();
    bg->key.assign(solvers, solvers + n);
    bg->bufs = batch_bufs(solvers, n);
    const int T = solvers[0]->T;
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    std::vector<BatchLaunchGroup> groups = batch_groups(solvers, n);
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int i = 0; i < n && e == hipSuccess; ++i) e = plan_iterations(solvers[i], T, cap);
        if (e == hipSuccess) e = enqueue_batch(groups, solvers, n, T, dim, cap);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
        bg->graph = graph;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(BSGD_E_DEVICE, "batched graph capture: %s", hipGetErrorString(e));
    out = std::move(bg);
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_step_batch(bsgd_solver* const* solvers, int32_t n, int32_t n_iters, void* stream)
{
    if (!solvers || n < 1 || n > 65536) return fail(BSGD_E_INVALID_ARG, "need 1 <= n <= 65536 solvers");
    if (n_iters < 0 || n_iters > (1 << 20)) return fail(BSGD_E_INVALID_ARG, "n_iters must be in [0, 2^20]");
    hipStream_t st = (hipStream_t)stream;
    const int dim = solvers[0] ? solvers[0]->g->dim : 0;
    for (int i = 0; i < n; ++i) {
        bsgd_solver* s = solvers[i];
        if (!s) return fail(BSGD_E_INVALID_ARG, "solver %d is NULL", i);
        if (s->failed) return fail(BSGD_E_STATE, "solver %d is in a failed state", i);
        if (s->st != st) return fail(BSGD_E_INVALID_ARG, "solver %d was created on another stream", i);
        if (s->g->dim != dim) return fail(BSGD_E_INVALID_ARG, "a batch mixes 2D and 3D solves");
        if (s->auto_mu) return fail(BSGD_E_UNSUPPORTED, "solver %d tunes its step length; step it alone", i);
        if (s->subdet) return fail(BSGD_E_UNSUPPORTED, "solver %d keeps sub-detector memories; step it alone", i);
        for (int j = 0; j < i; ++j)
            if (solvers[j] == s) return fail(BSGD_E_INVALID_ARG, "solver %d appears twice", i);
    }
    if (n_iters == 0) return BSGD_OK;
    auto mark_failed = [&](bsgd_status e) {
        for (int i = 0; i < n; ++i) solvers[i]->failed = true;
        return e;
    };
    for (int i = 0; i < n; ++i) {  // the caller may have changed x since the last call
        const hipError_t he = refresh_xT(solvers[i], st);
        if (he != hipSuccess) return mark_failed(fail(BSGD_E_DEVICE, "transpose of x: %s", hipGetErrorString(he)));
    }
    // one effective epoch from an epoch boundary of every solver, graphs allowed: replay
    // (or capture) the set's graph
    bool graph_ok = true;
    const int T = solvers[0]->T;
    for (int i = 0; i < n && graph_ok; ++i) {
        const bsgd_solver* s = solvers[i];
        graph_ok = s->graphs && !s->prof && s->T == T && n_iters == T && s->k % T == 0 &&
                   (!(s->o.tv_lambda > 0) || T % s->tv_every == 0);
    }
    if (graph_ok) {
        // buffers first (a reallocation would invalidate a captured graph)
        for (int i = 0; i < n; ++i) {
            bsgd_status stt = ensure_sched(solvers[i], T);
            if (stt != BSGD_OK) return mark_failed(stt);
        }
        const std::vector<bsgd_solver*> key(solvers, solvers + n);
        BatchGraph* bg = nullptr;
        bool capture = false;
        {
            std::lock_guard<std::mutex> lock(g_bg_mu);
            for (size_t i = 0; i < g_bg.size(); ++i)
                if (g_bg[i]->key == key) {
                    if (g_bg[i]->bufs != batch_bufs(solvers, n)) {
                        g_bg.erase(g_bg.begin() + i);  // a buffer moved since the capture
                        break;
                    }
                    std::unique_ptr<BatchGraph> hit = std::move(g_bg[i]);
                    g_bg.erase(g_bg.begin() + i);
                    g_bg.push_back(std::move(hit));
                    bg = g_bg.back().get();
                    break;
                }
            if (!bg) {
                capture = g_bg_last == key;
                g_bg_last = key;
            }
        }
        if (bg || capture) {
            for (int i = 0; i < n; ++i) {
                bsgd_status stt = upload_iterations(solvers[i], T, st);
                if (stt != BSGD_OK) return mark_failed(stt);
            }
            if (!bg) {
                std::unique_ptr<BatchGraph> fresh;
                bsgd_status stt = capture_batch_graph(solvers, n, dim, fresh);
                if (stt != BSGD_OK) return mark_failed(stt);
                std::lock_guard<std::mutex> lock(g_bg_mu);
                if (g_bg.size() >= BATCH_GRAPHS_KEPT) g_bg.erase(g_bg.begin());
                g_bg.push_back(std::move(fresh));
                bg = g_bg.back().get();
            }
            hipError_t he = hipGraphLaunch(bg->exec, st);
            if (he != hipSuccess) return mark_failed(fail(BSGD_E_DEVICE, "batched graph launch: %s", hipGetErrorString(he)));
            for (int i = 0; i < n; ++i) {
                solvers[i]->k += n_iters;
                mark_use(solvers[i], st);
            }
            return BSGD_OK;
        }
    }
    for (int i = 0; i < n; ++i) {
        bsgd_status stt = upload_iterations(solvers[i], n_iters, st);
        if (stt == BSGD_OK) {
            hipError_t he = plan_iterations(solvers[i], n_iters, st);
            if (he != hipSuccess) stt = fail(BSGD_E_DEVICE, "plan: %s", hipGetErrorString(he));
        }
        if (stt != BSGD_OK) return mark_failed(stt);
    }
    std::vector<BatchLaunchGroup> groups = batch_groups(solvers, n);
    hipError_t he = enqueue_batch(groups, solvers, n, n_iters, dim, st);
    if (he != hipSuccess) return mark_failed(fail(BSGD_E_DEVICE, "batched launch: %s", hipGetErrorString(he)));
    for (int i = 0; i < n; ++i) {
        solvers[i]->k += n_iters;
        mark_use(solvers[i], st);
    }
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_counts(const bsgd_solver* s, int64_t* iters_done, int32_t* rows, int32_t* blocks,
                                          int32_t* epoch_iters)
{
    if (!s) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    if (iters_done) *iters_done = s->k;
    if (rows) *rows = s->R;
    if (blocks) *blocks = s->B;
    if (epoch_iters) *epoch_iters = s->T;
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_last_schedule(const bsgd_solver* sc, int32_t* n_out, int32_t* rows,
                                                 int32_t* blocks, int16_t* draws, size_t draws_bytes)
{
    if (!sc) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    bsgd_solver* s = const_cast<bsgd_solver*>(sc);
    const int n = s->last_n;
    if (n_out) *n_out = n;
    const SchedLayout& L = s->L;
    for (int it = 0; it < n; ++it) {
        const int32_t* rec = s->last_sched.data() + (size_t)it * L.stride;
        if (rows) std::copy(rec + L.off_rows(), rec + L.off_rows() + L.R, rows + (size_t)it * L.R);
        if (blocks) std::copy(rec + L.off_blocks(), rec + L.off_blocks() + L.B, blocks + (size_t)it * L.B);
    }
    if (draws) {
        const size_t cnt = (size_t)n * s->maxv * s->B;
        if (draws_bytes < cnt * sizeof(int16_t)) return fail(BSGD_E_INVALID_ARG, "draws buffer too small");
        if (!s->im) {
            std::fill(draws, draws + cnt, (int16_t)-2);
        } else {
            std::vector<int8_t> tmp(cnt);
            HIP_TRY(hipStreamSynchronize(s->st));
            HIP_TRY(hipMemcpy(tmp.data(), s->draws.p, cnt, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < cnt; ++i) draws[i] = tmp[i];
        }
    }
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_state(const bsgd_solver* s, int32_t which, float* out, size_t bytes)
{
    if (!s || !out) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    const DevBuf* src = nullptr;
    size_t need = 0;
    if (which == 0) {
        src = &s->gsum;
        need = (size_t)s->g->n_vox * sizeof(float);
    } else if (which == 1) {
        if (s->subdet) return fail(BSGD_E_INVALID_ARG, "a solver with sub-detector memories keeps no g_hat");
        src = &s->ghat;
        need = (size_t)s->g->M * s->g->n_vox * sizeof(float);
    } else if (which == 2) {
        src = &s->z;
        need = (size_t)s->g->z_floats * sizeof(float);
    } else if (which == 3) {
        if (!s->subdet) return fail(BSGD_E_INVALID_ARG, "the solver keeps no sub-detector memories");
        src = &s->rho;
        need = (size_t)s->g->z_floats * sizeof(float);
    } else {
        return fail(BSGD_E_INVALID_ARG, "unknown state %d", which);
    }
    if (bytes < need) return fail(BSGD_E_INVALID_ARG, "state needs %zu bytes", need);
    HIP_TRY(hipMemcpyAsync(out, src->p, need, hipMemcpyDeviceToDevice, s->st));
    mark_use(s, s->st);
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_set_profiling(bsgd_solver* s, int32_t on)
{
    if (!s) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    s->prof = on != 0;
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solver_kernel_times(bsgd_solver* s, double* ms_out, int64_t* launches_out)
{
    if (!s) return fail(BSGD_E_INVALID_ARG, "solver is NULL");
    HIP_TRY(hipStreamSynchronize(s->st));
    for (auto& p : s->pending) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        s->ms[p.first] += ms;
        s->ev_pool.push_back(p.second.first);
        s->ev_pool.push_back(p.second.second);
    }
    s->pending.clear();
    for (int i = 0; i < KID_COUNT; ++i) {
        if (ms_out) ms_out[i] = s->ms[i];
        if (launches_out) launches_out[i] = s->launches[i];
    }
    return BSGD_OK;
}

// ||A^T (y - A x)|| with scratch buffers: ty [n_rays], tg [n_vox].
static bsgd_status normal_residual(const bsgd_geometry* g, const float* y, const float* x, float* ty, float* tg,
                                   double* partials, double* dout, double* host_out, hipStream_t st, double* out)
{
    HIP_TRY(launch_fp_full(g->dg, g->d_all_views.as<int32_t>(), g->d.n_views, -1, x, ty, 0, st));
    HIP_TRY(launch_sub(y, ty, ty, g->n_rays, st));
    HIP_TRY(launch_bp_full(g->dg, g->d_all_views.as<int32_t>(), g->d.n_views, -1, ty, tg, 1.0f, 0, st));
    int np = 0;
    HIP_TRY(launch_sumsq(tg, g->n_vox, partials, &np, st));
    HIP_TRY(launch_sum_partials(partials, np, dout, st));
    HIP_TRY(hipMemcpyAsync(host_out, dout, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(*host_out);
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_normal_residual(bsgd_solver* const* solvers, int32_t n, int32_t relative, double* out,
                                            void* stream)
{
    if (!solvers || !out || n < 1 || n > 65536) return fail(BSGD_E_INVALID_ARG, "need 1 <= n <= 65536 solvers and out");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        if (!solvers[i]) return fail(BSGD_E_INVALID_ARG, "solver %d is NULL", i);
        if (solvers[i]->st != st) return fail(BSGD_E_INVALID_ARG, "solver %d was created on another stream", i);
    }
    // norm_out slots: [2] = ||A^T (y - A x)||^2, [3] = ||A^T y||^2 (first relative call)
    for (int i = 0; i < n; ++i) {
        bsgd_solver* s = solvers[i];
        const bsgd_geometry* g = s->g;
        if (!s->nr_ty.p) {
            HIP_TRY(s->nr_ty.alloc((size_t)g->n_rays * sizeof(float)));
            HIP_TRY(s->nr_tg.alloc((size_t)g->n_vox * sizeof(float)));
        }
        double* dout = s->norm_out.as<double>();
        double* part = s->partials.as<double>();
        float* ty = s->nr_ty.as<float>();
        float* tg = s->nr_tg.as<float>();
        const int32_t* views = g->d_all_views.as<int32_t>();
        int np = 0;
        if (relative && s->nr_ref < 0.0) {
            HIP_TRY(launch_fill(tg, 0.0f, g->n_vox, st));
            HIP_TRY(launch_bp_full(g->dg, views, g->d.n_views, -1, s->y, tg, 1.0f, 0, st));
            HIP_TRY(launch_sumsq(tg, g->n_vox, part, &np, st));
            HIP_TRY(launch_sum_partials(part, np, dout + 3, st));
        }
        HIP_TRY(launch_fp_full(g->dg, views, g->d.n_views, -1, s->x, ty, 0, st));
        HIP_TRY(launch_sub(s->y, ty, ty, g->n_rays, st));
        HIP_TRY(launch_bp_full(g->dg, views, g->d.n_views, -1, ty, tg, 1.0f, 0, st));
        HIP_TRY(launch_sumsq(tg, g->n_vox, part, &np, st));
        HIP_TRY(launch_sum_partials(part, np, dout + 2, st));
        HIP_TRY(hipMemcpyAsync(s->norm_host + 2, dout + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        bsgd_solver* s = solvers[i];
        if (relative && s->nr_ref < 0.0) s->nr_ref = std::sqrt(s->norm_host[3]);
        const double v = std::sqrt(s->norm_host[2]);
        out[i] = relative ? v / std::max(s->nr_ref, 1e-300) : v;
    }
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_normal_residual_async(bsgd_solver* const* solvers, int32_t n, double* out_sq,
                                                  void* stream)
{
    if (!solvers || !out_sq || n < 1 || n > 65536) return fail(BSGD_E_INVALID_ARG, "need 1 <= n <= 65536 solvers and out_sq");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        if (!solvers[i]) return fail(BSGD_E_INVALID_ARG, "solver %d is NULL", i);
        if (solvers[i]->st != st) return fail(BSGD_E_INVALID_ARG, "solver %d was created on another stream", i);
    }
    for (int i = 0; i < n; ++i) {
        bsgd_solver* s = solvers[i];
        const bsgd_geometry* g = s->g;
        if (!s->nr_ty.p) {
            HIP_TRY(s->nr_ty.alloc((size_t)g->n_rays * sizeof(float)));
            HIP_TRY(s->nr_tg.alloc((size_t)g->n_vox * sizeof(float)));
        }
        if (!s->nr_out.p) HIP_TRY(s->nr_out.alloc(2 * sizeof(double)));
        double* dout = s->nr_out.as<double>();
        double* part = s->partials.as<double>();
        float* ty = s->nr_ty.as<float>();
        float* tg = s->nr_tg.as<float>();
        const int32_t* views = g->d_all_views.as<int32_t>();
        int np = 0;
        if (!s->nr_ref_dev) {
            HIP_TRY(launch_fill(tg, 0.0f, g->n_vox, st));
            HIP_TRY(launch_bp_full(g->dg, views, g->d.n_views, -1, s->y, tg, 1.0f, 0, st));
            HIP_TRY(launch_sumsq(tg, g->n_vox, part, &np, st));
            HIP_TRY(launch_sum_partials(part, np, dout + 1, st));
            s->nr_ref_dev = true;
        }
        HIP_TRY(launch_fp_full(g->dg, views, g->d.n_views, -1, s->x, ty, 0, st));
        HIP_TRY(launch_sub(s->y, ty, ty, g->n_rays, st));
        HIP_TRY(launch_bp_full(g->dg, views, g->d.n_views, -1, ty, tg, 1.0f, 0, st));
        HIP_TRY(launch_sumsq(tg, g->n_vox, part, &np, st));
        HIP_TRY(launch_sum_partials(part, np, dout, st));
        HIP_TRY(hipMemcpyAsync(out_sq + 2 * i, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        mark_use(s, st);
    }
    return BSGD_OK;
}

extern "C" bsgd_status bsgd_solve(const bsgd_geometry* g, const float* y, float* x, const bsgd_options* o, void* stream,
                                  int32_t* iters_out, double* resid_norm_out)
{
    bsgd_solver* s = nullptr;
    hipStream_t st = (hipStream_t)stream;
    bsgd_status stt = solver_create(g, y, x, o, st, &s);
    if (stt != BSGD_OK) return stt;
    const int epochs = o->max_effective_epochs > 0 ? o->max_effective_epochs : 1;
    const int check = o->check_every > 0 ? o->check_every : 1;
    DevBuf ty, tg;
    g->bind(ty);
    g->bind(tg);
    double ref = 0.0;
    if (o->tol > 0) {
        if (ty.alloc((size_t)g->n_rays * sizeof(float)) != hipSuccess ||
            tg.alloc((size_t)g->n_vox * sizeof(float)) != hipSuccess) {
            delete s;
            return fail(BSGD_E_OUT_OF_MEMORY, "no memory for the stopping-rule scratch");
        }
        // ||A^T y||: the normal residual at x = 0
        HIP_TRY(launch_fill(tg.as<float>(), 0.0f, g->n_vox, st));
        HIP_TRY(launch_bp_full(g->dg, g->d_all_views.as<int32_t>(), g->d.n_views, -1, y, tg.as<float>(), 1.0f, 0, st));
        int np = 0;
        HIP_TRY(launch_sumsq(tg.as<float>(), g->n_vox, s->partials.as<double>(), &np, st));
        HIP_TRY(launch_sum_partials(s->partials.as<double>(), np, s->norm_out.as<double>(), st));
        HIP_TRY(hipMemcpyAsync(s->norm_host, s->norm_out.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ref = std::sqrt(*s->norm_host);
    }
    for (int e = 0; e < epochs; ++e) {
        stt = bsgd_step(s, s->T, nullptr);
        if (stt != BSGD_OK) break;
        if (o->tol > 0 && ((e + 1) % check == 0 || e + 1 == epochs)) {
            double nr = 0.0;
            stt = normal_residual(g, y, x, ty.as<float>(), tg.as<float>(), s->partials.as<double>(),
                                  s->norm_out.as<double>(), s->norm_host, st, &nr);
            if (stt != BSGD_OK) break;
            if (!std::isfinite(nr)) {
                stt = fail(BSGD_E_DIVERGED, "normal residual is not finite");
                break;
            }
            if (ref > 0 && nr / ref <= o->tol) break;
        }
    }
    double rn = 0.0;
    if (stt == BSGD_OK) stt = bsgd_step(s, 0, &rn);
    if (stt == BSGD_OK) {
        if (iters_out) *iters_out = (int32_t)s->k;
        if (resid_norm_out) *resid_norm_out = rn;
    }
    delete s;
    return stt;
}

// ------------------------------------------------------------ allocation-free normal residual

// Scratch of bsgd_normal_residual_noalloc: the residual y - A x, the back projection
// A^T (y - A x), the reduction partials and the final sum, in one file-scope device
// array that every GPU the library runs on holds until the process ends. Host code
// never uses the array's name as a device address: the address is looked up once
// per device with hipGetSymbolAddress and kept in scratch_dev.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_PARTIALS = 4096;  // launch_sumsq never uses more partials
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

static bsgd_status scratch_address(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(BSGD_E_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(BSGD_E_DEVICE, "no device address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return BSGD_OK;
}

static size_t round_up_256(size_t b) { return (b + 255) & ~size_t(255); }

extern "C" size_t bsgd_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

extern "C" bsgd_status bsgd_normal_residual_noalloc(const bsgd_geometry* g, const float* y, const float* x,
                                                    double* out, void* stream)
{
    if (!g || !y || !x || !out) return fail(BSGD_E_INVALID_ARG, "NULL argument");
    const size_t ty_bytes = round_up_256((size_t)g->n_rays * sizeof(float));
    const size_t tg_bytes = round_up_256((size_t)g->n_vox * sizeof(float));
    const size_t part_bytes = round_up_256((size_t)NOALLOC_MAX_PARTIALS * sizeof(double));
    const size_t need = ty_bytes + tg_bytes + part_bytes + 256;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(BSGD_E_INVALID_ARG, "geometry needs %zu bytes of scratch (rays %lld, voxels %lld); the limit is %zu",
                    need, (long long)g->n_rays, (long long)g->n_vox, NOALLOC_SCRATCH_BYTES);
    void* base = nullptr;
    bsgd_status stt = scratch_address(&base);
    if (stt != BSGD_OK) return stt;
    unsigned char* b = static_cast<unsigned char*>(base);
    float* ty = reinterpret_cast<float*>(b);
    float* tg = reinterpret_cast<float*>(b + ty_bytes);
    double* part = reinterpret_cast<double*>(b + ty_bytes + tg_bytes);
    double* dout = reinterpret_cast<double*>(b + ty_bytes + tg_bytes + part_bytes);
    hipStream_t st = (hipStream_t)stream;
    // every scratch word read below is first written on this stream: the forward
    // projection writes every ray, the back projection of all blocks every voxel,
    // k_sumsq every partial it reports and k_sum_partials the sum
    const int32_t* views = g->d_all_views.as<int32_t>();
    HIP_TRY(launch_fp_full(g->dg, views, g->d.n_views, -1, x, ty, 0, st));
    HIP_TRY(launch_sub(y, ty, ty, g->n_rays, st));
    HIP_TRY(launch_bp_full(g->dg, views, g->d.n_views, -1, ty, tg, 1.0f, 0, st));
    int np = 0;
    HIP_TRY(launch_sumsq(tg, g->n_vox, part, &np, st));
    if (np > NOALLOC_MAX_PARTIALS) return fail(BSGD_E_DEVICE, "reduction used %d partials", np);
    HIP_TRY(launch_sum_partials(part, np, dout, st));
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(&v, dout, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(v);
    return BSGD_OK;
}
