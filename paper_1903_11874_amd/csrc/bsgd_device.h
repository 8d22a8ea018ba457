// Device-side geometry records and the per-(ray, voxel) arithmetic shared by all
// kernels. The forward projector (ray-driven Siddon walk), the back projector
// (voxel-driven slab test) and the importance-weight pass all evaluate a_ij with
// the same formulas in the same block-local frame, so the back projection is the
// exact transpose of the forward projection up to FP32 summation order.
//
// Frames and precision: every ray is re-anchored per column block. Its point is
// taken on the plane through the block centre perpendicular to the central ray,
// at lateral offset lambda = (k - kc) au + bu (and (l - lc) av + bv along z) from
// the block centre; au, bu, kc are derived in FP64 on the host per (view, block).
// The direction is the unnormalised source-to-pixel vector (a, b[, v]) with
// |(a, b, v)| = sqrt(sdd^2 + u^2 + v^2) (fan / cone) or the unit vector (parallel).
// Its reciprocals and length are precomputed in FP64 per (view, pixel column) and
// per pixel row (ray tables), so every kernel reads identical values. The walk
// parameter t is in units of that length; a_ij = dt * |d|. All plane positions are
// block-local, X_i = i v - h, exact in FP32. A direction component that is exactly
// zero is stored as an infinite reciprocal; such an axis is never crossed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsgd {

enum : int32_t { KIND_PARALLEL_2D = 0, KIND_FAN_2D = 1, KIND_CONE_3D = 2 };

// One (view, column block) pair. 64 bytes.
struct PairInfo {
    int32_t u0, u1, v0, v1;  // detector footprint of the block, half-open pixel ranges
    int64_t zoff;            // first float of this pair's z slot, laid out [l - v0][k - u0]
    float au, bu, av, bv;    // lateral ray offsets at the block-centre plane (mm)
    int32_t kc, lc;          // anchor pixel indices for the offsets
    float cu;                // block centre . e_u (mm)
    float depth;             // source to block-centre plane distance (mm); 0 for parallel
    float cz;                // block centre z (mm)
    int32_t pad;
};

// Work record of one (view slot, block slot) pair of one iteration, written by the
// plan kernel: the pixel range to process (footprint, restricted to the drawn
// sub-detector), the z addressing and the ray anchors of the pair. 80 bytes.
struct PairWork {
    int32_t k0, k1, l0, l1;  // half-open pixel ranges; empty when k1 <= k0
    int64_t zbase;           // z index of pixel (k, l) is zbase + l * zw + k
    int32_t zw;              // footprint width (row stride of the z slot)
    int32_t view;
    float au, bu, av, bv;    // as in PairInfo
    int32_t kc, lc;
    float cu, depth, cz;
    float c, s;              // cos, sin of the view angle
    int32_t pad;
};

// One column block. 48 bytes.
struct BlockInfo {
    int32_t x0, y0, z0;      // first voxel
    int32_t nbx, nby, nbz;   // voxels per axis
    float hx, hy, hz;        // half extents (mm)
    float pad0, pad1, pad2;
};

struct DevGeom {
    int32_t kind, dim;
    int32_t nx, ny, nz;
    float vx, vy, vz;
    int32_t n_views, nu, nv;
    float du, dv, sod, sdd;
    int32_t N, bx, by, bz;
    int32_t su, sv, S;
    const float2* cs;          // [n_views] (cos, sin)
    const PairInfo* pairs;     // [n_views][N]
    const BlockInfo* blocks;   // [N]
    const float4* raydir;      // [n_views][nu]: 1/a, 1/b, |(a,b)|^2 (cone) or |d| (2D), unused
    const float2* rayv;        // [nv]: 1/v, v^2 (cone only)
    int32_t fp_chunk;          // views per workgroup of the LDS forward projector (tuning)
    int32_t fp_split;          // lanes per 2D ray in the LDS forward projector: 1, 2 or 4 (tuning)
    int32_t fp_wpp;            // waves per (view, block) pair of the global-memory forward projector
    int32_t bp_split;          // waves of a 2D back-projection tile, each a share of the views: 2, 4 or 8 (tuning)
    // 2D chord tables: per (view, pixel) the unit normal (nx, ny) of the ray, xi with
    // n . p = lambda xi for the ray's anchor point p, and the trapezoid of the chord
    // length through one voxel as a function of the signed distance of the voxel
    // centre from the ray: plateau half-width w1, support half-width w2, plateau
    // length lmax and flank slope lmax / (w2 - w1). Per view: kspan, the candidate
    // half-range in pixels times the depth of the centre (fan) or in pixels (parallel),
    // first of one voxel, then of two x-adjacent voxels as one 2 x 1 rectangle.
    const float4* raynorm;     // [n_views][nu]: nx, ny, xi, unused
    const float4* raytrap;     // [n_views][nu]: w1, w2, lmax, slope
    const float* kspan;        // [2][n_views]: one voxel, two voxels
    // Pixel-major index of z: ray p = view * nu * nv + l * nu + k has the z slots
    // cov_idx[cov_off[p] .. cov_off[p + 1]), one per column block whose footprint holds
    // the pixel, blocks ascending. NULL when z has 2^32 or more slots (the residual
    // rebuild then tests the footprint rectangles itself).
    const uint32_t* cov_off;   // [n_views * nu * nv + 1]
    const uint32_t* cov_idx;   // [z_floats]
    // 3D back projection: largest pixel rectangle (columns, rows) a workgroup tile
    // projects to in one view, the size of its LDS staging per view; 0 = no staging
    int32_t bp3_kmax, bp3_lmax;
    int32_t bp3_steep;  // some ray's chord through a voxel column can meet two z planes
    // every block spans fewer than 2^29 voxels of x, so the global 3D forward walk's
    // offsets of nonzero steps fit the byte range (below 2^31) of a buffer load
    int32_t fp_buf;
};

// Sub-detector s covers u in [k0, k1), v in [l0, l1).
__device__ __forceinline__ void subdet_range(const DevGeom& G, int s, int& k0, int& k1, int& l0, int& l1)
{
    int a = s % G.su, b = s / G.su;
    k0 = (a * G.nu) / G.su;
    k1 = ((a + 1) * G.nu) / G.su;
    l0 = (b * G.nv) / G.sv;
    l1 = ((b + 1) * G.nv) / G.sv;
}

// Ray (k, l) of a view, in the block-local frame of pair P.
struct Ray {
    float p[3];    // point on the block-centre plane, block-local (mm)
    float inv[3];  // reciprocal of the direction (inf for a zero component)
    float len;     // |d| (mm per unit t)
};

// steps of the 3D / 2D wave-uniform walks whose loads are issued together
constexpr int WALK_UNROLL = 8;
constexpr int WALK2_UNROLL = 4;

__device__ __forceinline__ bool axis_fixed(float inv) { return __builtin_isinf(inv); }

// P is a PairInfo or a PairWork (same anchor fields).
template <int DIM, class Anchor>
__device__ __forceinline__ void make_ray(const DevGeom& G, int view, float c, float s, const Anchor& P, int k,
                                         int l, Ray& R)
{
    const float lu = fmaf((float)(k - P.kc), P.au, P.bu);
    R.p[0] = -lu * s;
    R.p[1] = lu * c;
    const float4 T = G.raydir[(int64_t)view * G.nu + k];
    R.inv[0] = T.x;
    R.inv[1] = T.y;
    if (DIM == 3) {
        R.p[2] = fmaf((float)(l - P.lc), P.av, P.bv);
        const float2 V = G.rayv[l];
        R.inv[2] = V.x;
        R.len = __builtin_amdgcn_sqrtf(T.z + V.y);
    } else {
        R.len = T.z;
    }
}

__device__ __forceinline__ float plane_pos(int i, float v, float h) { return fmaf((float)i, v, -h); }

__device__ __forceinline__ float plane_t(int i, float v, float h, float p, float inv)
{
    return (plane_pos(i, v, h) - p) * inv;
}

// Entry voxel index along one axis at parameter tlo, exact with respect to plane_t,
// the next crossing parameter and the step direction.
__device__ __forceinline__ void walk_axis_init(const Ray& R, int a, int n, float h, float vs, float tlo, int& idx,
                                               int& step, float& tn)
{
    const bool fixed = axis_fixed(R.inv[a]);
    // estimate only: the loops below make the index exact with respect to plane_t
    const float pos = fixed ? R.p[a] : fmaf(tlo, __builtin_amdgcn_rcpf(R.inv[a]), R.p[a]);
    float fi = floorf((pos + h) * __builtin_amdgcn_rcpf(vs));
    fi = fminf(fmaxf(fi, 0.0f), (float)(n - 1));
    int i = (int)fi;
    step = 0;
    tn = INFINITY;
    if (fixed) {
        while (i < n - 1 && R.p[a] >= plane_pos(i + 1, vs, h)) ++i;
        while (i > 0 && R.p[a] < plane_pos(i, vs, h)) --i;
    } else if (R.inv[a] > 0.0f) {
        while (i < n - 1 && plane_t(i + 1, vs, h, R.p[a], R.inv[a]) <= tlo) ++i;
        while (i > 0 && plane_t(i, vs, h, R.p[a], R.inv[a]) > tlo) --i;
        step = 1;
        tn = plane_t(i + 1, vs, h, R.p[a], R.inv[a]);
    } else {
        while (i > 0 && plane_t(i, vs, h, R.p[a], R.inv[a]) <= tlo) --i;
        while (i < n - 1 && plane_t(i + 1, vs, h, R.p[a], R.inv[a]) > tlo) ++i;
        step = -1;
        tn = plane_t(i, vs, h, R.p[a], R.inv[a]);
    }
    idx = i;
}

// Ray-driven Siddon walk through one block. visit(off, dt) is called for every
// voxel the ray crosses, in order, with the voxel's offset off = iz sz + iy sy + ix
// in the block's storage and the parameter length dt >= 0 (dt = 0 at exact corner
// crossings; ties cross the lowest axis first). The step is branch free: the
// crossed axis' operands are selected and its next plane parameter is computed
// with the same plane_t formula the back projector's slab test uses.
template <int DIM, class Visit>
__device__ __forceinline__ void walk_block(const Ray& R, const int (&nb)[3], const float (&h)[3],
                                           const float (&vs)[3], int sy, int sz, Visit&& visit)
{
    float tlo = -INFINITY, thi = INFINITY;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float X0 = -h[a];
        float Xn = plane_pos(nb[a], vs[a], h[a]);
        if (!axis_fixed(R.inv[a])) {
            float t0 = (X0 - R.p[a]) * R.inv[a];
            float t1 = (Xn - R.p[a]) * R.inv[a];
            tlo = fmaxf(tlo, fminf(t0, t1));
            thi = fminf(thi, fmaxf(t0, t1));
        } else if (!(X0 <= R.p[a] && R.p[a] < Xn)) {
            return;
        }
    }
    if (!(tlo < thi)) return;

    int ix, iy, iz = 0, sx, sy_, sz_ = 0;
    float tx, ty, tz = INFINITY;
    walk_axis_init(R, 0, nb[0], h[0], vs[0], tlo, ix, sx, tx);
    walk_axis_init(R, 1, nb[1], h[1], vs[1], tlo, iy, sy_, ty);
    if (DIM == 3) walk_axis_init(R, 2, nb[2], h[2], vs[2], tlo, iz, sz_, tz);
    // next plane index per axis (the exit plane of the current voxel)
    int px = ix + (sx > 0), py = iy + (sy_ > 0), pz = iz + (sz_ > 0);
    int off = iz * sz + iy * sy + ix;

    float t = tlo;
    const int max_steps = nb[0] + nb[1] + (DIM == 3 ? nb[2] : 0) + 2;
    for (int it = 0; it < max_steps; ++it) {
        const bool cx = (tx <= ty) && (DIM == 2 || tx <= tz);
        const bool cy = !cx && (DIM == 2 || ty <= tz);
        const float tm = cx ? tx : (cy ? ty : tz);
        visit(off, tm - t);
        t = tm;
        // advance the crossed axis
        const int st = cx ? sx : (cy ? sy_ : sz_);
            if (DIM == 2) {
            ix += cx ? sx : 0;
            iy += cx ? 0 : sy_;
            px += cx ? sx : 0;
            py += cx ? 0 : sy_;
            off += cx ? sx : sy_ * sy;
            const bool out = cx ? (ix < 0 || ix >= nb[0]) : (iy < 0 || iy >= nb[1]);
            if (st == 0 || out) break;
            const int kk = cx ? px : py;
            const float pv = cx ? vs[0] : vs[1], ph = cx ? h[0] : h[1];
            const float pp = cx ? R.p[0] : R.p[1], pi = cx ? R.inv[0] : R.inv[1];
            const float tnew = plane_t(kk, pv, ph, pp, pi);
            tx = cx ? tnew : tx;
            ty = cx ? ty : tnew;
        } else {
            const bool cz = !cx && !cy;
            ix += cx ? sx : 0;
            iy += cy ? sy_ : 0;
            iz += cz ? sz_ : 0;
            px += cx ? sx : 0;
            py += cy ? sy_ : 0;
            pz += cz ? sz_ : 0;
            off += cx ? sx : (cy ? sy_ * sy : sz_ * sz);
            const bool out = cx ? (ix < 0 || ix >= nb[0]) : (cy ? (iy < 0 || iy >= nb[1]) : (iz < 0 || iz >= nb[2]));
            if (st == 0 || out) break;
            const int kk = cx ? px : (cy ? py : pz);
            const float pv = cx ? vs[0] : (cy ? vs[1] : vs[2]);
            const float ph = cx ? h[0] : (cy ? h[1] : h[2]);
            const float pp = cx ? R.p[0] : (cy ? R.p[1] : R.p[2]);
            const float pi = cx ? R.inv[0] : (cy ? R.inv[1] : R.inv[2]);
            const float tnew = plane_t(kk, pv, ph, pp, pi);
            tx = cx ? tnew : tx;
            ty = cy ? tnew : ty;
            tz = cz ? tnew : tz;
        }
    }
}

// Parameter interval [tlo, thi) of a 2D ray inside a block (same slab formula as
// walk_block); false when the ray misses the block.
__device__ __forceinline__ bool slab_2d(const Ray& R, const int (&nb)[3], const float (&h)[3], const float (&vs)[3],
                                        float& tlo, float& thi)
{
    tlo = -INFINITY;
    thi = INFINITY;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const float X0 = -h[a];
        const float Xn = plane_pos(nb[a], vs[a], h[a]);
        if (!axis_fixed(R.inv[a])) {
            const float t0 = (X0 - R.p[a]) * R.inv[a];
            const float t1 = (Xn - R.p[a]) * R.inv[a];
            tlo = fmaxf(tlo, fminf(t0, t1));
            thi = fminf(thi, fmaxf(t0, t1));
        } else if (!(X0 <= R.p[a] && R.p[a] < Xn)) {
            return false;
        }
    }
    return tlo < thi;
}

// Forward-projection walk of a 2D ray over the parameter range [t0, t1) inside one
// block (t0, t1 within the slab): returns the sum over the pixels crossed of
// (parameter length) * value(off), off = iy sy + ix. The starting pixel, the first
// crossing per axis and the Siddon order (ties cross x first) are those of
// walk_block. The m-th later crossing of an axis is fmaf(m, v |inv|, t_first): one
// FMA per axis and step, with an error relative to the chord rather than to |inv|
// (an affine form in the plane index would cancel badly for near-axis rays). No
// bounds tests: the walk ends at t1. A crossing rounded to just below the block's
// exit can step one pixel past the block; the offset is clamped into the block, and
// that pixel's length is a few ulps of t.
template <class Load>
__device__ __forceinline__ float walk_2d_range(const Ray& R, const int (&nb)[3], const float (&h)[3],
                                               const float (&vs)[3], int sy, float t0, float t1, Load&& load)
{
    if (!(t0 < t1)) return 0.0f;
    int ix, iy, sx, sy_;
    float tx0, ty0;
    walk_axis_init(R, 0, nb[0], h[0], vs[0], t0, ix, sx, tx0);
    walk_axis_init(R, 1, nb[1], h[1], vs[1], t0, iy, sy_, ty0);
    const float ax = axis_fixed(R.inv[0]) ? 0.0f : vs[0] * fabsf(R.inv[0]);
    const float ay = axis_fixed(R.inv[1]) ? 0.0f : vs[1] * fabsf(R.inv[1]);
    float mx = 0.0f, my = 0.0f, tx = tx0, ty = ty0;
    const int dox = sx, doy = sy_ * sy;
    const unsigned last = (unsigned)((nb[1] - 1) * sy + nb[0] - 1);
    int off = iy * sy + ix;
    float t = t0, acc = 0.0f;
    const int max_steps = nb[0] + nb[1] + 2;
    // WALK2_UNROLL steps per round, loads issued together; steps past the exit have
    // zero length (t stays at t1) and clamped offsets, so they add exact zeros
    for (int it = 0; it < max_steps; it += WALK2_UNROLL) {
        unsigned o[WALK2_UNROLL];
        float dt[WALK2_UNROLL], v[WALK2_UNROLL];
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) {
            const bool cx = tx <= ty;
            const float tm = fminf(fminf(tx, ty), t1);
            // zero-length steps (past the exit) read the block's first pixel
            o[u] = tm > t ? min((unsigned)off, last) : 0u;
            dt[u] = tm - t;
            t = tm;
            off += cx ? dox : doy;
            mx += cx ? 1.0f : 0.0f;
            my += cx ? 0.0f : 1.0f;
            tx = fmaf(mx, ax, tx0);
            ty = fmaf(my, ay, ty0);
        }
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) v[u] = load(o[u]);
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) acc = fmaf(dt[u], v[u], acc);
        if (t >= t1) break;
    }
    return acc;
}

// Largest int over the 64 lanes of a wave (all lanes must be active).
__device__ __forceinline__ int wave_max_int(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// walk_2d_range with a wave-uniform trip count, for callers whose 64 lanes are all
// active: each lane bounds its pixel count by the plane crossings its parameter range
// can hold, the wave loops to the largest bound on a scalar counter, and a lane past
// its end adds zero-length steps (tm = t = t1). No per-lane exit, so no exec-mask
// bookkeeping per step. live = false gives 0. Offsets are iy sy + ix sx_ from the
// block's first pixel (sx_ = 1 for x stored fastest, the y extent for x stored y fastest).
template <class Load>
__device__ __forceinline__ float walk_2d_range_wave(const Ray& R, const int (&nb)[3], const float (&h)[3],
                                                    const float (&vs)[3], int sx_, int sy, float t0, float t1,
                                                    bool live, Load&& load)
{
    live = live && (t0 < t1);
    int ix = 0, iy = 0, sx = 0, sy_ = 0;
    float tx0 = INFINITY, ty0 = INFINITY;
    if (live) {
        walk_axis_init(R, 0, nb[0], h[0], vs[0], t0, ix, sx, tx0);
        walk_axis_init(R, 1, nb[1], h[1], vs[1], t0, iy, sy_, ty0);
    } else {
        t0 = t1 = 0.0f;
    }
    const float ax = (live && !axis_fixed(R.inv[0])) ? vs[0] * fabsf(R.inv[0]) : 0.0f;
    const float ay = (live && !axis_fixed(R.inv[1])) ? vs[1] * fabsf(R.inv[1]) : 0.0f;
    // pixels visited <= crossings of each axis in (t0, t1) + 1, plus one step past
    // the exit by rounding; fminf also maps inf/NaN (fixed axis, empty range) away
    const float cap = (float)(nb[0] + nb[1] + 2);
    const float span = t1 - t0;
    const float nxf = ax > 0.0f ? fminf(floorf(span * __builtin_amdgcn_rcpf(ax)), cap) : 0.0f;
    const float nyf = ay > 0.0f ? fminf(floorf(span * __builtin_amdgcn_rcpf(ay)), cap) : 0.0f;
    const int n = live ? (int)fminf(nxf + nyf + 4.0f, cap) : 0;
    const int n_wave = wave_max_int(n);
    float mx = 0.0f, my = 0.0f, tx = tx0, ty = ty0;
    const int dox = sx * sx_, doy = sy_ * sy;
    const unsigned last = (unsigned)((nb[1] - 1) * sy + (nb[0] - 1) * sx_);
    int off = iy * sy + ix * sx_;
    float t = t0, acc = 0.0f;
    // WALK2_UNROLL steps at a time, as in walk_3d_range_wave: offsets and lengths, then
    // the loads, then the FMAs in step order
    int it = 0;
    for (; it + WALK2_UNROLL <= n_wave; it += WALK2_UNROLL) {
        unsigned o[WALK2_UNROLL];
        float dt[WALK2_UNROLL], v[WALK2_UNROLL];
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) {
            const bool cx = tx <= ty;
            const float tm = fminf(fminf(tx, ty), t1);
            o[u] = min((unsigned)off, last);
            dt[u] = tm - t;
            t = tm;
            off += cx ? dox : doy;
            mx += cx ? 1.0f : 0.0f;
            my += cx ? 0.0f : 1.0f;
            tx = fmaf(mx, ax, tx0);
            ty = fmaf(my, ay, ty0);
        }
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) v[u] = load(o[u]);
#pragma unroll
        for (int u = 0; u < WALK2_UNROLL; ++u) acc = fmaf(dt[u], v[u], acc);
    }
    for (; it < n_wave; ++it) {
        const bool cx = tx <= ty;
        const float tm = fminf(fminf(tx, ty), t1);
        acc = fmaf(tm - t, load(tm > t ? min((unsigned)off, last) : 0u), acc);
        t = tm;
        off += cx ? dox : doy;
        mx += cx ? 1.0f : 0.0f;
        my += cx ? 0.0f : 1.0f;
        tx = fmaf(mx, ax, tx0);
        ty = fmaf(my, ay, ty0);
    }
    return acc;
}

// Parameter interval [tlo, thi) of a 3D ray inside a block (same slab formula as
// walk_block); false when the ray misses the block.
__device__ __forceinline__ bool slab_3d(const Ray& R, const int (&nb)[3], const float (&h)[3], const float (&vs)[3],
                                        float& tlo, float& thi)
{
    tlo = -INFINITY;
    thi = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float X0 = -h[a];
        const float Xn = plane_pos(nb[a], vs[a], h[a]);
        if (!axis_fixed(R.inv[a])) {
            const float t0 = (X0 - R.p[a]) * R.inv[a];
            const float t1 = (Xn - R.p[a]) * R.inv[a];
            tlo = fmaxf(tlo, fminf(t0, t1));
            thi = fminf(thi, fmaxf(t0, t1));
        } else if (!(X0 <= R.p[a] && R.p[a] < Xn)) {
            return false;
        }
    }
    return tlo < thi;
}

// The 3D form of walk_2d_range_wave: Siddon order with ties crossing x, then y, then
// z (as walk_block); the m-th later crossing of an axis is fmaf(m, v |inv|, t_first);
// wave-uniform trip count from the crossings each lane's range can hold. load(off)
// gets the offset off = iz sz + iy sy + ix sx from the block's first voxel, in the units
// of the strides passed (elements or bytes; sx is one element for x stored fastest, the
// y extent of x for the copy stored y fastest); for
// steps of zero length (past a ray's exit, or a lane without a ray) off may lie outside
// the block or wrap, and load must then return any finite value (it is multiplied by
// zero). All 64 lanes must be active.
template <class Load>
__device__ __forceinline__ float walk_3d_range_wave(const Ray& R, const int (&nb)[3], const float (&h)[3],
                                                    const float (&vs)[3], int sx_, int sy, int sz, float t0,
                                                    float t1, bool live, Load&& load)
{
    live = live && (t0 < t1);
    int ix = 0, iy = 0, iz = 0, sx = 0, sy_ = 0, sz_ = 0;
    float tx0 = INFINITY, ty0 = INFINITY, tz0 = INFINITY;
    if (live) {
        walk_axis_init(R, 0, nb[0], h[0], vs[0], t0, ix, sx, tx0);
        walk_axis_init(R, 1, nb[1], h[1], vs[1], t0, iy, sy_, ty0);
        walk_axis_init(R, 2, nb[2], h[2], vs[2], t0, iz, sz_, tz0);
    } else {
        t0 = t1 = 0.0f;
    }
    const float ax = (live && !axis_fixed(R.inv[0])) ? vs[0] * fabsf(R.inv[0]) : 0.0f;
    const float ay = (live && !axis_fixed(R.inv[1])) ? vs[1] * fabsf(R.inv[1]) : 0.0f;
    const float az = (live && !axis_fixed(R.inv[2])) ? vs[2] * fabsf(R.inv[2]) : 0.0f;
    const float cap = (float)(nb[0] + nb[1] + nb[2] + 2);
    const float span = t1 - t0;
    const float nxf = ax > 0.0f ? fminf(floorf(span * __builtin_amdgcn_rcpf(ax)), cap) : 0.0f;
    const float nyf = ay > 0.0f ? fminf(floorf(span * __builtin_amdgcn_rcpf(ay)), cap) : 0.0f;
    const float nzf = az > 0.0f ? fminf(floorf(span * __builtin_amdgcn_rcpf(az)), cap) : 0.0f;
    const int n = live ? (int)fminf(nxf + nyf + nzf + 5.0f, cap) : 0;
    const int n_wave = wave_max_int(n);
    float mx = 0.0f, my = 0.0f, mz = 0.0f, tx = tx0, ty = ty0, tz = tz0;
    const int dox = sx * sx_, doy = sy_ * sy, doz = sz_ * sz;
    int off = iz * sz + iy * sy + ix * sx_;
    float t = t0, acc = 0.0f;
    // WALK_UNROLL steps at a time: their voxel offsets and lengths first (the stepping
    // never depends on loaded values), then the gathers back to back, then the FMAs in
    // step order (the same sum as one step at a time). The crossing axis is the one whose
    // next crossing equals the minimum (ties: x, then y, then z).
    int it = 0;
    for (; it + WALK_UNROLL <= n_wave; it += WALK_UNROLL) {
        unsigned o[WALK_UNROLL];
        float dt[WALK_UNROLL], v[WALK_UNROLL];
#pragma unroll
        for (int u = 0; u < WALK_UNROLL; ++u) {
            const float m3 = fminf(fminf(tx, ty), tz);
            const bool cx = tx == m3;
            const bool cy = !cx && ty == m3;
            const float tm = fminf(m3, t1);
            // a step of zero length (past the ray's exit) reads the block's first voxel,
            // so finished lanes share one cache line instead of wandering along their rays
            o[u] = tm > t ? (unsigned)off : 0u;
            dt[u] = tm - t;
            t = tm;
            off += cx ? dox : (cy ? doy : doz);
            mx += cx ? 1.0f : 0.0f;
            my += cy ? 1.0f : 0.0f;
            mz += (cx || cy) ? 0.0f : 1.0f;
            tx = fmaf(mx, ax, tx0);
            ty = fmaf(my, ay, ty0);
            tz = fmaf(mz, az, tz0);
        }
#pragma unroll
        for (int u = 0; u < WALK_UNROLL; ++u) v[u] = load(o[u]);
#pragma unroll
        for (int u = 0; u < WALK_UNROLL; ++u) acc = fmaf(dt[u], v[u], acc);
    }
    for (; it < n_wave; ++it) {
        const float m3 = fminf(fminf(tx, ty), tz);
        const bool cx = tx == m3;
        const bool cy = !cx && ty == m3;
        const float tm = fminf(m3, t1);
        acc = fmaf(tm - t, load(tm > t ? (unsigned)off : 0u), acc);
        t = tm;
        off += cx ? dox : (cy ? doy : doz);
        mx += cx ? 1.0f : 0.0f;
        my += cy ? 1.0f : 0.0f;
        mz += (cx || cy) ? 0.0f : 1.0f;
        tx = fmaf(mx, ax, tx0);
        ty = fmaf(my, ay, ty0);
        tz = fmaf(mz, az, tz0);
    }
    return acc;
}

// Whole chord of a 2D ray through one block.
template <class Load>
__device__ __forceinline__ float walk_2d_sum(const Ray& R, const int (&nb)[3], const float (&h)[3],
                                             const float (&vs)[3], int sy, Load&& load)
{
    float tlo, thi;
    if (!slab_2d(R, nb, h, vs, tlo, thi)) return 0.0f;
    return walk_2d_range(R, nb, h, vs, sy, tlo, thi, load);
}

// Length parameter of ray R inside block-local voxel (ix, iy, iz): the slab test
// with the same plane formula as walk_block. Returns dt (0 when the ray misses).
template <int DIM>
__device__ __forceinline__ float voxel_dt(const Ray& R, const int (&ix)[3], const float (&h)[3], const float (&vs)[3])
{
    float te = -INFINITY, tx = INFINITY;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (!axis_fixed(R.inv[a])) {
            float t0 = plane_t(ix[a], vs[a], h[a], R.p[a], R.inv[a]);
            float t1 = plane_t(ix[a] + 1, vs[a], h[a], R.p[a], R.inv[a]);
            te = fmaxf(te, fminf(t0, t1));
            tx = fminf(tx, fmaxf(t0, t1));
        } else {
            if (!(plane_pos(ix[a], vs[a], h[a]) <= R.p[a] && R.p[a] < plane_pos(ix[a] + 1, vs[a], h[a])))
                return 0.0f;
        }
    }
    return fmaxf(tx - te, 0.0f);
}

// One axis of voxel_dt's slab test for a ray with coordinate p and reciprocal
// direction inv on that axis through voxel index i: narrows [te, tx], or clears hit
// when the ray runs parallel to the axis outside the voxel.
__device__ __forceinline__ void slab_axis(float p, float inv, int i, float v, float h, float& te, float& tx, bool& hit)
{
    if (!axis_fixed(inv)) {
        const float t0 = plane_t(i, v, h, p, inv);
        const float t1 = plane_t(i + 1, v, h, p, inv);
        te = fmaxf(te, fminf(t0, t1));
        tx = fminf(tx, fmaxf(t0, t1));
    } else if (!(plane_pos(i, v, h) <= p && p < plane_pos(i + 1, v, h))) {
        hit = false;
    }
}

// Exact length of a line through an axis-aligned rectangle (2D voxel) as a function
// of the signed distance delta of the rectangle centre from the line: lmax on the
// plateau |delta| <= w1, falling linearly to 0 at |delta| = w2 (a trapezoid).
__device__ __forceinline__ float chord_2d(float delta, const float4& trap)
{
    // the slope is finite (capped on the host), so the product is never NaN and the
    // clamp to [0, lmax] is one median-of-three
    return __builtin_amdgcn_fmed3f((trap.y - fabsf(delta)) * trap.w, 0.0f, trap.z);
}

// chord_2d on a per-ray record {w2, slope, lmax, r}: the same operations on the same
// values, so the same bits.
__device__ __forceinline__ float chord_2d_rec(float delta, const float4& rec)
{
    return __builtin_amdgcn_fmed3f((rec.x - fabsf(delta)) * rec.y, 0.0f, rec.z);
}

// SplitMix64 output function and the counter-based draws (same definition as the
// host runtime's selection streams).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash3(uint64_t seed, uint64_t stream, uint64_t k1, uint64_t k2, uint64_t k3)
{
    uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull * (1ull + stream));
    h = mix64(h ^ k1);
    h = mix64(h ^ k2);
    return mix64(h ^ k3);
}

}  // namespace bsgd
