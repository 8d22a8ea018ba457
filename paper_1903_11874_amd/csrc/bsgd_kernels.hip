// HIP kernels for gfx950 (CDNA4, wave64) of the BSGD hot path:
//   forward projection of sampled (view, block) pairs      Algorithm 1/2, z refresh
//   residual rebuild r = y - sum_j z^j on the sampled rows  Algorithm 1, residual line
//   matched back projection fused with the block step      Algorithm 1, g_hat / g / x lines
//   sub-detector draws and importance weights              Algorithm 2, Sec. II-A
//   TV proximal step                                        Algorithm 4
//   deterministic wave64 reductions for residual norms      Algorithm 3 (norm of r)
// Projection is a sparse gather, not a dense contraction, so nothing here uses
// MFMA. No kernel uses global atomics; every sum has a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "bsgd_device.h"
#include "bsgd_kernels.h"

namespace bsgd {

namespace {

constexpr int WG = 256;
constexpr float SHADOW_EPS = 1e-3f;  // candidate-range margin of the voxel shadow, in pixels
constexpr int BP_AHEAD = 2;          // 2D back projection: candidates whose gathers are issued together

// Workgroups go to the 8 XCDs round-robin (workgroup id mod 8), and each XCD has its
// own L2. Renumbering so that consecutive logical workgroups run on one XCD keeps the
// workgroups of one column block (same image tile, same work records) in one L2:
// logical = first logical id of XCD (id mod 8) + (id div 8). A bijection of [0, n).
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_local(int id, int n)
{
    const int per = n / N_XCD, rem = n % N_XCD;
    const int x = id % N_XCD, s = id / N_XCD;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + s;
}

// The (x, y) of a 2D grid in the renumbered order (x fastest, as dispatched).
__device__ __forceinline__ void xcd_grid2(int& bx, int& by)
{
    const int gx = (int)gridDim.x;
    const int l = xcd_local((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    bx = l % gx;
    by = l / gx;
}

__device__ __forceinline__ void block_dims(const DevGeom& G, const BlockInfo& B, int (&nb)[3], float (&h)[3],
                                           float (&vs)[3])
{
    nb[0] = B.nbx;
    nb[1] = B.nby;
    nb[2] = B.nbz;
    h[0] = B.hx;
    h[1] = B.hy;
    h[2] = B.hz;
    vs[0] = G.vx;
    vs[1] = G.vy;
    vs[2] = G.vz;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide (256 threads) double sum in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((lds[0] + lds[1]) + (lds[2] + lds[3]));
    __syncthreads();
    return r;
}

// Rectangle of pixels processed for one (view, block) pair: footprint, intersected
// with the drawn sub-detector when s >= 0.
__device__ __forceinline__ void pair_range(const DevGeom& G, const PairInfo& P, int s, int& k0, int& k1, int& l0,
                                           int& l1)
{
    k0 = P.u0;
    k1 = P.u1;
    l0 = P.v0;
    l1 = P.v1;
    if (s >= 0) {
        int a0, a1, b0, b1;
        subdet_range(G, s, a0, a1, b0, b1);
        k0 = max(k0, a0);
        k1 = min(k1, a1);
        l0 = max(l0, b0);
        l1 = min(l1, b1);
    }
}

// Forward projection of ray (k, l) through block j of view v: sum_i a_i x_i (mm * x).
// xb points at the block's first voxel with row stride sy and slice stride sz (global
// memory or an LDS copy of the block).
template <int DIM, class Anchor, class Ptr>
__device__ __forceinline__ float fp_ray_block(const DevGeom& G, int view, float c, float s, const Anchor& P,
                                              const BlockInfo& B, int k, int l, Ptr xb, int64_t sy, int64_t sz)
{
    Ray R;
    make_ray<DIM>(G, view, c, s, P, k, l, R);
    int nb[3];
    float h[3], vs[3];
    block_dims(G, B, nb, h, vs);
    if (DIM == 2) return walk_2d_sum(R, nb, h, vs, (int)sy, [&](unsigned off) { return xb[off]; }) * R.len;
    float acc = 0.0f;
    walk_block<DIM>(R, nb, h, vs, (int)sy, (int)sz, [&](int off, float dt) { acc = fmaf(dt, xb[off], acc); });
    return acc * R.len;
}

// Load base[byte_off / sizeof(T)] with a 32-bit byte offset (a uniform base stays in
// scalar registers; the offset is one vector register).
template <class T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Candidate pixel range [klo, khi] of a 2D voxel centre (qx, qy), block-local, in one
// view: the pixels within kc -/+ span of the projection of the centre (kspan / depth for
// a fan, kspan for parallel rays; kspan bounds the chord's support), clipped to [k0, k1).
// which = 1 takes the span of two x-adjacent voxels and (qx, qy) the centre of their
// shared edge. For a fan the bound is exact for any convex body: a ray at distance d
// from the centre meets the detector d |ray| / depth away from the centre's projection,
// and it can cross the body only while d is within the body's support half-width.
template <class Anchor>
__device__ __forceinline__ void bp2d_range(const DevGeom& G, int view, float c, float s, const Anchor& P, float qx,
                                           float qy, int k0, int k1, int& klo, int& khi, int which = 0)
{
    const float w = fmaf(qy, c, -(qx * s)) + P.cu;
    const float ku = 0.5f * (float)(G.nu - 1);
    const float inv_du = __builtin_amdgcn_rcpf(G.du);
    float kc, span;
    if (G.kind == KIND_PARALLEL_2D) {
        kc = fmaf(w, inv_du, ku);
        span = G.kspan[which * G.n_views + view];
    } else {
        const float rdep = __builtin_amdgcn_rcpf(P.depth - fmaf(qx, c, qy * s));
        kc = fmaf(G.sdd * w * rdep, inv_du, ku);
        span = G.kspan[which * G.n_views + view] * rdep;
    }
    klo = (int)ceilf(fminf(fmaxf(kc - span - SHADOW_EPS, (float)k0), (float)k1));
    khi = min(k1 - 1, (int)floorf(fmaxf(fminf(kc + span + SHADOW_EPS, (float)k1), (float)k0 - 1.0f)));
}

// 2D back projection of one view into two x-adjacent voxels (li and li + one voxel in
// x; the second only when b_ok): the candidates of both are walked once, so each
// candidate's ray normal and {w2, slope, lmax, r} record (PACKED) or trapezoid and
// residual are gathered once for two voxels. A candidate outside a voxel's own range
// lies outside its chord's support (the range is conservative), so it adds an exact
// zero.
template <bool PACKED, class Anchor>
__device__ __forceinline__ void bp_voxel_pair_view_2d(const DevGeom& G, int view, float c, float s, const Anchor& P,
                                                      const int (&li)[3], bool b_ok, const float (&h)[3],
                                                      const float (&vs)[3], int k0, int k1,
                                                      const float* __restrict__ src, float& acc_a, float& acc_b)
{
    const float qxa = plane_pos(li[0], vs[0], h[0]) + 0.5f * vs[0];
    const float qxb = plane_pos(li[0] + 1, vs[0], h[0]) + 0.5f * vs[0];
    const float qy = plane_pos(li[1], vs[1], h[1]) + 0.5f * vs[1];
    // candidates: the shadow of voxel a, or of the two voxels as one 2 x 1 rectangle about
    // their shared edge (its own support half-width; the bound is the same)
    int lo, hi;
    if (b_ok)
        bp2d_range(G, view, c, s, P, plane_pos(li[0] + 1, vs[0], h[0]), qy, k0, k1, lo, hi, 1);
    else
        bp2d_range(G, view, c, s, P, qxa, qy, k0, k1, lo, hi, 0);
    const float4* nrm = G.raynorm + (int64_t)view * G.nu;
    const float4* trp = G.raytrap + (int64_t)view * G.nu;
    const float4* rec = reinterpret_cast<const float4*>(src);
    float4 n[BP_AHEAD], t[BP_AHEAD];
    float r[BP_AHEAD];
#pragma unroll
    for (int i = 0; i < BP_AHEAD; ++i) {
        if (lo + i <= hi) {
            const uint32_t kk = (uint32_t)(lo + i);
            n[i] = ld_off(nrm, kk * 16u);
            if constexpr (PACKED) {
                t[i] = ld_off(rec, kk * 16u);
            } else {
                t[i] = ld_off(trp, kk * 16u);
                r[i] = ld_off(src, kk * 4u);
            }
        }
    }
    const float lam0 = fmaf((float)(lo - P.kc), P.au, P.bu);
    auto add = [&](const float4& nk, const float4& tk, float rk, float lam) {
        const float base = fmaf(nk.y, qy, -(lam * nk.z));
        const float da = fmaf(nk.x, qxa, base), db = fmaf(nk.x, qxb, base);
        if constexpr (PACKED) {
            acc_a = fmaf(chord_2d_rec(da, tk), tk.w, acc_a);
            acc_b = fmaf(chord_2d_rec(db, tk), tk.w, acc_b);
        } else {
            acc_a = fmaf(chord_2d(da, tk), rk, acc_a);
            acc_b = fmaf(chord_2d(db, tk), rk, acc_b);
        }
    };
#pragma unroll
    for (int i = 0; i < BP_AHEAD; ++i)
        if (lo + i <= hi) add(n[i], t[i], PACKED ? 0.0f : r[i], fmaf((float)i, P.au, lam0));
    for (int k = lo + BP_AHEAD; k <= hi; ++k) {
        const uint32_t kk = (uint32_t)k;
        const float4 nk = ld_off(nrm, kk * 16u);
        const float lam = fmaf((float)(k - lo), P.au, lam0);
        if constexpr (PACKED)
            add(nk, ld_off(rec, kk * 16u), 0.0f, lam);
        else
            add(nk, ld_off(trp, kk * 16u), ld_off(src, kk * 4u), lam);
    }
}

// ------------------------------------------------------------ geometry statistics

// One wave per (view, block) pair: for every sub-detector s, w = sum over its rays
// of sum_i a_i^2 and the number of positive-length segments.
template <int DIM>
__global__ __launch_bounds__(WG) void k_geom_stats(DevGeom G, double* __restrict__ w, long long* __restrict__ nnz)
{
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (WG / 64) + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int n_pairs = G.n_views * G.N;
    if (wave >= n_pairs) return;
    const int v = wave / G.N, j = wave % G.N;
    const PairInfo P = G.pairs[wave];
    const BlockInfo B = G.blocks[j];
    const float2 cs = G.cs[v];
    int nb[3];
    float h[3], vs[3];
    block_dims(G, B, nb, h, vs);
    for (int sd = 0; sd < G.S; ++sd) {
        int k0, k1, l0, l1;
        pair_range(G, P, sd, k0, k1, l0, l1);
        const int wk = k1 - k0, wl = l1 - l0;
        const int n = (wk > 0 && wl > 0) ? wk * wl : 0;
        double acc = 0.0;
        long long cnt = 0;
        for (int q = lane; q < n; q += 64) {
            const int k = k0 + q % wk, l = l0 + q / wk;
            Ray R;
            make_ray<DIM>(G, v, cs.x, cs.y, P, k, l, R);
            float s2 = 0.0f;
            int ns = 0;
            walk_block<DIM>(R, nb, h, vs, 0, 0, [&](int, float dt) {
                s2 = fmaf(dt, dt, s2);
                ns += dt > 0.0f;
            });
            acc += (double)s2 * (double)R.len * (double)R.len;
            cnt += ns;
        }
        acc = wave_sum(acc);
        cnt = wave_sum_ll(cnt);
        if (lane == 0) {
            const int64_t o = ((int64_t)v * G.S + sd) * G.N + j;
            w[o] = acc;
            nnz[o] = cnt;
        }
    }
}

// ------------------------------------------------------------ iteration plan (draws + work records)

// One thread per (iteration, block slot, view slot): draw the sub-detector of
// Algorithm 2 when sampling is on (counter-based: hash of (seed, IM stream, k,
// view, block), first s whose running sum of q exceeds bounded(hash, sum q)), and
// write the pair's work record. Draws are stored [it][view slot][block slot] for
// export; records [it][block slot][view slot] so that a block's views are contiguous.
__global__ __launch_bounds__(WG) void k_plan(DevGeom G, const int32_t* __restrict__ sched, SchedLayout L,
                                             int it0, unsigned long long seed,
                                             const uint32_t* __restrict__ q, long long im_until,
                                             int8_t* __restrict__ draws, PairWork* __restrict__ work)
{
    // x: (block slot, view slot) of one iteration; y: iteration it0 + blockIdx.y
    const int per_it = L.maxv * L.B;
    const int rem = (int)blockIdx.x * WG + (int)threadIdx.x;
    if (rem >= per_it) return;
    const int it = it0 + (int)blockIdx.y;
    const int64_t gid = (int64_t)it * per_it + rem;
    const int b = rem / L.maxv, a = rem - b * L.maxv;
    const int32_t* S_ = sched + (int64_t)it * L.stride;
    PairWork W;
    W.k0 = W.k1 = W.l0 = W.l1 = 0;
    W.zbase = 0;
    W.zw = 0;
    W.view = 0;
    W.au = W.bu = W.av = W.bv = 0.0f;
    W.kc = W.lc = 0;
    W.cu = W.depth = W.cz = 0.0f;
    W.c = W.s = 0.0f;
    W.pad = 0;
    int8_t dr = DRAW_SKIP;
    if (a < S_[0]) {
        const int v = S_[L.off_views() + a];
        const int j = S_[L.off_blocks() + b];
        int sd = -2;
        const uint64_t kit = (uint64_t)(uint32_t)S_[L.off_k()] | ((uint64_t)(uint32_t)S_[L.off_k() + 1] << 32);
        if (q && (im_until <= 0 || (long long)kit < im_until)) {
            unsigned long long total = 0;
            for (int t = 0; t < G.S; ++t) total += q[((int64_t)v * G.S + t) * G.N + j];
            sd = DRAW_SKIP;
            if (total > 0) {
                const uint64_t kk = (uint64_t)(uint32_t)S_[L.off_k()] | ((uint64_t)(uint32_t)S_[L.off_k() + 1] << 32);
                const uint64_t hsh = hash3(seed, 4ull, kk, (uint64_t)v, (uint64_t)j);
                const uint64_t u = __umul64hi(hsh, total);
                unsigned long long accq = 0;
                sd = G.S - 1;
                for (int t = 0; t < G.S; ++t) {
                    accq += q[((int64_t)v * G.S + t) * G.N + j];
                    if (accq > u) {
                        sd = t;
                        break;
                    }
                }
            }
            dr = (int8_t)sd;
        } else if (q) {
            dr = (int8_t)-2;  // unbiased tail: every ray of the view
        }
        if (sd != DRAW_SKIP) {
            const PairInfo P = G.pairs[(int64_t)v * G.N + j];
            pair_range(G, P, sd, W.k0, W.k1, W.l0, W.l1);
            if (W.k1 <= W.k0 || W.l1 <= W.l0) W.k0 = W.k1 = W.l0 = W.l1 = 0;
            W.zw = P.u1 - P.u0;
            W.zbase = P.zoff - (int64_t)P.v0 * W.zw - P.u0;
            W.view = v;
            W.au = P.au;
            W.bu = P.bu;
            W.av = P.av;
            W.bv = P.bv;
            W.kc = P.kc;
            W.lc = P.lc;
            W.cu = P.cu;
            W.depth = P.depth;
            W.cz = P.cz;
            const float2 cs = G.cs[v];
            W.c = cs.x;
            W.s = cs.y;
        }
    }
    if (draws) draws[(int64_t)it * per_it + (int64_t)a * L.B + b] = dr;
    work[gid] = W;
}

// ------------------------------------------------------------ solver: forward projection

// G.fp_wpp waves per (view slot, block slot) pair: z^j = A_{rows}^{J_j} x_{J_j} on the
// pair's range. The range is cut into patches of 8 x 8 pixels (2D: 64 x 1), and wave w of
// a pair walks patches w, w + fp_wpp, ... one lane per pixel; every lane runs every
// round (lanes off the range are dead), so the walk's trip count is wave-uniform. A
// square patch keeps the chord lengths of a wave's rays close (a row of 64 pixels spans
// the footprint from edge to centre), so fewer steps are wasted on the longest ray. x is
// gathered from global memory (blocks too large for LDS).
template <int DIM>
__device__ __forceinline__ void fp_global_body(const DevGeom& G, const PairWork* __restrict__ work, SchedLayout L,
                                               const int32_t* __restrict__ blocks_sel, const float* __restrict__ x,
                                               const float* __restrict__ xT, float* __restrict__ z, int wave,
                                               int lane)
{
    const int wpp = max(1, G.fp_wpp);
    const int pair = wave / wpp, w = wave - pair * wpp;
    if (pair >= L.maxv * L.B) return;
    const int b = pair / L.maxv;
    const PairWork W = work[pair];
    const int wk = W.k1 - W.k0, wl = W.l1 - W.l0;
    if (wk <= 0 || wl <= 0) return;
    constexpr int PX = DIM == 3 ? 16 : 64, PY = 64 / PX;
    const int npx = (wk + PX - 1) / PX, n_patch = npx * ((wl + PY - 1) / PY);
    if (n_patch <= w) return;
    const BlockInfo B = G.blocks[blocks_sel[b]];
    // rays running closer to x than to y sit side by side in y: they gather from the copy
    // of x stored y fastest ([z][x][y]), where a patch's neighbouring rays read
    // neighbouring floats (x stored x fastest would put each on its own cache line)
    const bool tr = xT != nullptr && fabsf(W.c) >= fabsf(W.s);
    const int64_t xbase = tr ? ((int64_t)B.z0 * G.nx + B.x0) * (int64_t)G.ny + B.y0
                             : ((int64_t)B.z0 * G.ny + B.y0) * (int64_t)G.nx + B.x0;
    const float* xb = (tr ? xT : x) + xbase;
    const int sx = tr ? G.ny : 1, sy = tr ? 1 : G.nx, sz = G.nx * G.ny;
    int nb[3];
    float h[3], vs[3];
    block_dims(G, B, nb, h, vs);
    const unsigned last = (unsigned)((nb[2] - 1) * sz + (nb[1] - 1) * sy + (nb[0] - 1) * sx);
    const int64_t rem = ((int64_t)G.nx * G.ny * G.nz - xbase) * (int64_t)sizeof(float);
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void*)xb, (short)0, (int)min(rem, (int64_t)0x7fffffff), 0x00020000);
    const int rounds = (n_patch - w + wpp - 1) / wpp;
    for (int r = 0; r < rounds; ++r) {
        const int pt = w + wpp * r;
        const int kk = (pt % npx) * PX + lane % PX, ll = (pt / npx) * PY + lane / PX;
        const bool on = kk < wk && ll < wl;
        const int l = W.l0 + (on ? ll : 0), k = W.k0 + (on ? kk : 0);
        Ray R;
        make_ray<DIM>(G, W.view, W.c, W.s, W, k, l, R);
        float tlo = 0.0f, thi = 0.0f, acc;
        if (DIM == 2) {
            const bool hit = on && slab_2d(R, nb, h, vs, tlo, thi);
            acc = walk_2d_range_wave(R, nb, h, vs, sx, sy, tlo, thi, hit, [&](unsigned off) { return xb[off]; });
        } else {
            const bool hit = on && slab_3d(R, nb, h, vs, tlo, thi);
            if (G.fp_buf) {
                // raw buffer loads: the walk steps byte offsets from the block's first voxel
                // (strides in bytes) and the range ends with x, past which loads return 0
                acc = walk_3d_range_wave(R, nb, h, vs, 4 * sx, 4 * sy, 4 * sz, tlo, thi, hit, [&](unsigned off) {
                    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, off, 0, 0));
                });
            } else {
                acc = walk_3d_range_wave(R, nb, h, vs, sx, sy, sz, tlo, thi, hit,
                                         [&](unsigned off) { return xb[min(off, last)]; });
            }
        }
        if (on) z[W.zbase + (int64_t)l * W.zw + k] = acc * R.len;
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_fp_pairs(DevGeom G, const PairWork* __restrict__ work, SchedLayout L,
                                                 const int32_t* __restrict__ blocks_sel, const float* __restrict__ x,
                                                 const float* __restrict__ xT, float* __restrict__ z)
{
    const int wg = xcd_local((int)blockIdx.x, (int)gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(wg * (WG / 64) + (threadIdx.x >> 6));
    fp_global_body<DIM>(G, work, L, blocks_sel, x, xT, z, wave, threadIdx.x & 63);
}

// The copy of x stored y fastest: xT[(z nx + x) ny + y] = x[(z ny + y) nx + x], through a
// padded 32 x 32 LDS tile per (x tile, y tile, z).
__global__ __launch_bounds__(WG) void k_xy_transpose(const float* __restrict__ x, float* __restrict__ xT, int nx,
                                                     int ny)
{
    __shared__ float t[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int64_t zoff = (int64_t)blockIdx.z * nx * ny;
    const int c = threadIdx.x % 32, r0 = threadIdx.x / 32;
    for (int r = r0; r < 32; r += WG / 32)
        if (x0 + c < nx && y0 + r < ny) t[r][c] = x[zoff + (int64_t)(y0 + r) * nx + x0 + c];
    __syncthreads();
    for (int r = r0; r < 32; r += WG / 32)
        if (y0 + c < ny && x0 + r < nx) xT[zoff + (int64_t)(x0 + r) * ny + y0 + c] = t[c][r];
}

constexpr int FP_MAX_CHUNK = 16;
constexpr int FP_LDS_WG = 1024;  // threads per workgroup of the single-solve LDS forward projector
constexpr int FP_LDS_MAX_FLOATS = 16384;  // block copies up to 64 KB are staged in LDS; larger blocks read x from global memory

// Workgroup per (view chunk, block slot): the block's image tile is copied to LDS
// once and every ray of the chunk's pairs walks it there. Work items are the rays
// of all pairs of the chunk, flattened.
struct FpLds {
    PairWork pw[FP_MAX_CHUNK];
    int off[FP_MAX_CHUNK + 1];
};

template <int DIM, int TPB>
__device__ __forceinline__ void fp_lds_body(const DevGeom& G, const PairWork* __restrict__ work, SchedLayout L,
                                            const int32_t* __restrict__ blocks_sel, const float* __restrict__ x,
                                            float* __restrict__ z, int chunk, int bx, int by, float* xs, FpLds& sh)
{
    const int b = by;
    const int a_begin = bx * chunk;
    if (a_begin >= L.maxv) return;
    const int nch = min(chunk, L.maxv - a_begin);
    const PairWork* wb = work + (int64_t)b * L.maxv + a_begin;
    if (threadIdx.x < nch) sh.pw[threadIdx.x] = wb[threadIdx.x];
    const BlockInfo B = G.blocks[blocks_sel[b]];
    // 2D rows are padded by one float: at a given step, rays one pixel apart sit one
    // row apart, and an unpadded stride of nbx floats maps them to one LDS bank.
    const int rs = B.nbx + (DIM == 2 ? 1 : 0);
    const int plane = rs * B.nby;
    const int nvox_b = B.nbx * B.nby * B.nbz;
    if (B.nbx <= TPB) {
        // row by row: each thread keeps one column and steps over rows (one division
        // per thread instead of three per element)
        const int rpp = TPB / B.nbx;  // rows per pass
        const int col = (int)threadIdx.x % B.nbx, r0 = (int)threadIdx.x / B.nbx;
        const int rows = B.nby * B.nbz;
        if (r0 < rpp) {
            int iy = r0 % B.nby, iz = r0 / B.nby;
            const int dy = rpp % B.nby, dz = rpp / B.nby;
            for (int r = r0; r < rows; r += rpp) {
                xs[iz * plane + iy * rs + col] =
                    x[((int64_t)(B.z0 + iz) * G.ny + (B.y0 + iy)) * (int64_t)G.nx + (B.x0 + col)];
                iy += dy;
                iz += dz;
                if (iy >= B.nby) {
                    iy -= B.nby;
                    ++iz;
                }
            }
        }
    } else {
        for (int i = threadIdx.x; i < nvox_b; i += TPB) {
            const int ix = i % B.nbx, iy = (i / B.nbx) % B.nby, iz = i / (B.nbx * B.nby);
            xs[iz * plane + iy * rs + ix] =
                x[((int64_t)(B.z0 + iz) * G.ny + (B.y0 + iy)) * (int64_t)G.nx + (B.x0 + ix)];
        }
    }
    // the walk may step one pixel past an x face with a length of a few ulps; that
    // read lands in the padding column, which must hold a finite value
    if (DIM == 2)
        for (int iy = threadIdx.x; iy < B.nby; iy += TPB) xs[iy * rs + B.nbx] = 0.0f;
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
        for (int q = 0; q < nch; ++q) {
            sh.off[q] = off;
            off += max(0, sh.pw[q].k1 - sh.pw[q].k0) * max(0, sh.pw[q].l1 - sh.pw[q].l0);
        }
        sh.off[nch] = off;
    }
    __syncthreads();
    const int total = sh.off[nch];
    if (DIM == 2) {
        // S adjacent lanes per ray, each walking 1/S of the chord's parameter range;
        // the S partial sums are combined as (s0 + s1) + (s2 + s3), a fixed order.
        const int lg = G.fp_split >= 4 ? 2 : (G.fp_split >= 2 ? 1 : 0);
        const int S = 1 << lg;
        const float invS = 1.0f / (float)S;
        int nb[3];
        float h[3], vs[3];
        block_dims(G, B, nb, h, vs);
        // every thread runs every round (items past the end are dead lanes), so the
        // walk's wave-uniform trip count and the shuffles see all 64 lanes
        const int n_items = total << lg;
        const int rounds = (n_items + TPB - 1) / TPB;
        for (int rd = 0; rd < rounds; ++rd) {
            const int item = rd * TPB + (int)threadIdx.x;
            const bool on = item < n_items;
            const int ray = on ? (item >> lg) : 0, seg = item & (S - 1);
            // the pair holding this ray: the largest q with off[q] <= ray (empty pairs,
            // whose offsets repeat, are passed over), by bisection over the chunk
            int q = 0, qhi = nch - 1;
            while (q < qhi) {
                const int mid = (q + qhi + 1) >> 1;
                if (sh.off[mid] <= ray)
                    q = mid;
                else
                    qhi = mid - 1;
            }
            const PairWork& W = sh.pw[q];
            const int k = W.k0 + (ray - sh.off[q]);
            Ray R;
            make_ray<2>(G, W.view, W.c, W.s, W, k, W.l0, R);
            float tlo = 0.0f, thi = 0.0f;
            const bool hit = on && slab_2d(R, nb, h, vs, tlo, thi);
            const float span = thi - tlo;
            const float t0 = seg == 0 ? tlo : fmaf((float)seg * invS, span, tlo);
            const float t1 = seg == S - 1 ? thi : fmaf((float)(seg + 1) * invS, span, tlo);
            float acc = walk_2d_range_wave(R, nb, h, vs, 1, rs, t0, t1, hit, [&](unsigned off) { return xs[off]; });
            if (S >= 2) acc += __shfl_xor(acc, 1, 64);
            if (S >= 4) acc += __shfl_xor(acc, 2, 64);
            if (on && seg == 0) z[W.zbase + (int64_t)W.l0 * W.zw + k] = acc * R.len;
        }
        return;
    }
    for (int item = threadIdx.x; item < total; item += TPB) {
        int q = 0;
        while (sh.off[q + 1] <= item) ++q;
        const PairWork& W = sh.pw[q];
        const int r = item - sh.off[q];
        const int wk = W.k1 - W.k0;
        const int l = W.l0 + r / wk;
        const int k = W.k0 + (r - (l - W.l0) * wk);
        z[W.zbase + (int64_t)l * W.zw + k] =
            fp_ray_block<DIM>(G, W.view, W.c, W.s, W, B, k, l, xs, (int64_t)rs, (int64_t)plane);
    }
}

// Workgroup per (view chunk, block slot): the block's image tile is copied to LDS
// once and every ray of the chunk's pairs walks it there. Work items are the rays
// of all pairs of the chunk, flattened.
template <int DIM>
__global__ __launch_bounds__(FP_LDS_WG) void k_fp_pairs_lds(DevGeom G, const PairWork* __restrict__ work, SchedLayout L,
                                                     const int32_t* __restrict__ blocks_sel,
                                                     const float* __restrict__ x, float* __restrict__ z, int chunk)
{
    extern __shared__ float xs[];
    __shared__ FpLds sh;
    int bx, by;
    xcd_grid2(bx, by);
    fp_lds_body<DIM, FP_LDS_WG>(G, work, L, blocks_sel, x, z, chunk, bx, by, xs, sh);
}

// ------------------------------------------------------------ solver: residual rebuild

// Residual workgroup size: 64 threads in 2D, where one iteration has few rays and
// small workgroups spread them over every CU; 256 in 3D, where rays are plentiful and
// fewer, larger workgroups stage each view's rectangles fewer times.
__host__ __device__ constexpr int res_wg(int dim) { return dim == 3 ? 256 : 64; }

// r = y - sum_j z^j for every ray of one view (j ascending); the view's footprint
// rectangles are staged in LDS, with the bounding rectangle of each group of blocks
// that are consecutive in j (see res_group_size): a ray tests
// a group's blocks only when the group's rectangle contains it. The z offsets of the
// blocks containing the ray are first collected (per thread, in LDS) and then loaded
// back to back, so the gathers overlap; subtraction order stays ascending j.
// z offsets collected per thread before their gathers are issued (deeper in 2D, where
// LDS per workgroup is small)
__host__ __device__ constexpr int res_batch(int tpb) { return tpb == 64 ? 16 : 8; }

// one z slab per group in 3D; in 2D the blocks form one group (a row of blocks spans
// most of the detector, so a finer test prunes too little to pay for itself)
__host__ __device__ inline int res_group_size(const DevGeom& G) { return G.bz > 1 ? G.bx * G.by : G.N; }
__host__ __device__ inline int res_groups(const DevGeom& G)
{
    const int gs = res_group_size(G);
    return (G.N + gs - 1) / gs;
}

template <int RB>
__device__ __forceinline__ float resid_ray(const DevGeom& G, int v, int k, int l, const float* __restrict__ y,
                                           const float* __restrict__ z, const int4* rc, const long long* zo,
                                           const int4* grc, long long* cand, int per_view, int ray)
{
    float acc = y[(int64_t)v * per_view + ray];
    const int gs = res_group_size(G), ng = res_groups(G);
    int cnt = 0;
    for (int g = 0; g < ng; ++g) {
        const int4 b4 = grc[g];
        if (!(k >= b4.x && k < b4.y && l >= b4.z && l < b4.w)) continue;
        const int j1 = min(G.N, (g + 1) * gs);
        for (int j = g * gs; j < j1; ++j) {
            const int4 r4 = rc[j];
            if (k >= r4.x && k < r4.y && l >= r4.z && l < r4.w) {
                cand[cnt++] = zo[j] + (int64_t)(l - r4.z) * (r4.y - r4.x) + (k - r4.x);
                if (cnt == RB) {
                    float vals[RB];
#pragma unroll
                    for (int c = 0; c < RB; ++c) vals[c] = z[cand[c]];
#pragma unroll
                    for (int c = 0; c < RB; ++c) acc -= vals[c];
                    cnt = 0;
                }
            }
        }
    }
    for (int c0 = 0; c0 < cnt; c0 += 4) {
        float vals[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) vals[c] = (c0 + c < cnt) ? z[cand[c0 + c]] : 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c0 + c < cnt) acc -= vals[c];
    }
    return acc;
}

// r = y - sum_j z^j for ray p through the pixel-major z index, blocks ascending (the
// order of resid_ray, so both give the same bits). The index entries and z values of U
// blocks are gathered back to back.
template <int U>
__device__ __forceinline__ float resid_ray_idx(const DevGeom& G, int64_t p, const float* __restrict__ y,
                                               const float* __restrict__ z)
{
    const uint32_t o0 = G.cov_off[p], o1 = G.cov_off[p + 1];
    float acc = y[p];
    for (uint32_t e = o0; e < o1; e += U) {
        uint32_t id[U];
        float val[U];
#pragma unroll
        for (int c = 0; c < U; ++c) id[c] = (e + c < o1) ? G.cov_idx[e + c] : 0u;
#pragma unroll
        for (int c = 0; c < U; ++c) val[c] = (e + c < o1) ? z[id[c]] : 0.0f;
#pragma unroll
        for (int c = 0; c < U; ++c)
            if (e + c < o1) acc -= val[c];
    }
    return acc;
}

// Stage view v's footprint rectangles and z offsets, then the group bounding
// rectangles (empty footprints ignored; an empty group gets an empty rectangle).
__device__ __forceinline__ void stage_rects(const DevGeom& G, int v, int4* rc, long long* zo, int4* grc)
{
    const PairInfo* pv = G.pairs + (int64_t)v * G.N;
    for (int j = threadIdx.x; j < G.N; j += blockDim.x) {
        rc[j] = *reinterpret_cast<const int4*>(&pv[j].u0);
        zo[j] = pv[j].zoff;
    }
    __syncthreads();
    const int gs = res_group_size(G), ng = res_groups(G);
    if (ng == 1) {
        if (threadIdx.x == 0) grc[0] = make_int4(-0x7fffffff, 0x7fffffff, -0x7fffffff, 0x7fffffff);
        __syncthreads();
        return;
    }
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        int4 u = make_int4(0x7fffffff, -0x7fffffff, 0x7fffffff, -0x7fffffff);
        const int j1 = min(G.N, (g + 1) * gs);
        for (int j = g * gs; j < j1; ++j) {
            const int4 r4 = rc[j];
            if (r4.y <= r4.x || r4.w <= r4.z) continue;
            u.x = min(u.x, r4.x);
            u.y = max(u.y, r4.y);
            u.z = min(u.z, r4.z);
            u.w = max(u.w, r4.w);
        }
        if (u.y <= u.x) u = make_int4(0, 0, 0, 0);
        grc[g] = u;
    }
    __syncthreads();
}

// Dynamic LDS of the residual kernels: N int4 rectangles, the group rectangles (the
// 16-byte arrays first, so both stay 16-byte aligned), N 64-bit offsets, then
// res_batch candidate offsets per thread.
__host__ __device__ inline size_t resid_lds_bytes(const DevGeom& G, int threads)
{
    if (G.cov_off) return 0;  // the pixel-major index needs no staging
    return (size_t)G.N * (sizeof(int4) + sizeof(long long)) + (size_t)res_groups(G) * sizeof(int4) +
           (size_t)threads * res_batch(threads) * sizeof(long long);
}

// Residual of selected ray slot q (ray p of the geometry): a float in 3D; in 2D the
// record {w2, slope, lmax, r} the back projector gathers in one load.
__device__ __forceinline__ void store_resid(const DevGeom& G, float* __restrict__ r_sel, int64_t q, int64_t p, float r)
{
    if (G.dim == 2) {
        const float4 t = G.raytrap[p];
        reinterpret_cast<float4*>(r_sel)[q] = make_float4(t.y, t.w, t.z, r);
    } else {
        r_sel[q] = r;
    }
}

template <int TPB>
__device__ __forceinline__ void resid_body(const DevGeom& G, const int32_t* __restrict__ S_, SchedLayout L,
                                           const float* __restrict__ y, const float* __restrict__ z,
                                           float* __restrict__ r_sel, int bx, int by, int4* rc)
{
    int4* grc = rc + G.N;
    long long* zo = reinterpret_cast<long long*>(grc + res_groups(G));
    long long* cand = zo + G.N + threadIdx.x * res_batch(TPB);
    const int a = by;
    if (a >= S_[0]) return;
    const int v = S_[L.off_views() + a];
    const int per_view = G.nu * G.nv;
    if (G.cov_off) {  // uniform: the index replaces the rectangle tests
        const int ray = bx * TPB + threadIdx.x;
        if (ray < per_view)
            store_resid(G, r_sel, (int64_t)a * per_view + ray, (int64_t)v * per_view + ray,
                        resid_ray_idx<16>(G, (int64_t)v * per_view + ray, y, z));
        return;
    }
    stage_rects(G, v, rc, zo, grc);
    const int ray = bx * TPB + threadIdx.x;
    if (ray >= per_view) return;
    const int k = ray % G.nu, l = ray / G.nu;
    store_resid(G, r_sel, (int64_t)a * per_view + ray, (int64_t)v * per_view + ray,
                resid_ray<res_batch(TPB)>(G, v, k, l, y, z, rc, zo, grc, cand, per_view, ray));
}

template <int TPB>
__global__ __launch_bounds__(TPB) void k_resid(DevGeom G, const int32_t* __restrict__ S_, SchedLayout L,
                                                  const float* __restrict__ y, const float* __restrict__ z,
                                                  float* __restrict__ r_sel)
{
    extern __shared__ int4 rc[];
    int bx, by;
    xcd_grid2(bx, by);
    resid_body<TPB>(G, S_, L, y, z, r_sel, bx, by, rc);
}

// ------------------------------------------------------------ solver: back projection + step

// 2D: 64 lanes of two x-adjacent voxels per wave, each voxel's views interleaved over
// SPLIT waves (DevGeom::bp_split: 2, 4 or 8, a tuned launch shape) and the waves' partial
// sums added in a fixed order through LDS.
constexpr int BP_VOX = 64;
// waves of the standalone 2D back projection, and the default of the solver's. Measured on
// the 512^2 fan (2D back projection per iteration): one voxel per lane 36.1 / 30.5 / 30.9 us
// at 1 / 2 / 4 waves; two voxels per lane 29.4 / 24.0 / 24.6 us at 2 / 4 / 8 waves.
constexpr int BP_SPLIT_2D = 4;

// For each selected row block i: g_hat^i_new = 2 (A_{rows(i,j)}^{J_j})^T r;
// g += sum_i (g_hat^i_new - g_hat^i_old); g_hat^i = g_hat^i_new; then x += mu g.
// With SUB (gradient memory per (view, sub-detector, block), kept as the residual each
// ray had when its pair last ran): g += 2 (A_{rows}^{J_j})^T d with d = r - rho the
// change of those residuals, read from `src` in the z layout of each pair (k_subdet_delta
// wrote it); no g_hat. A voxel's update reads only r (or d), so voxels are independent
// (no atomics).
// 2D solver tiles: 16 x 8 voxels per wave, each lane two x-adjacent voxels.
constexpr int PAIR_TX = 16, PAIR_TY = 8;

// Lane vl's voxel pair in pair tile `tile` of block B: a at li, b one voxel further in x.
__device__ __forceinline__ void pair_tile_voxels(const BlockInfo& B, int tile, int vl, int (&li)[3], bool& tile_ok,
                                                 bool& a_ok, bool& b_ok)
{
    const int tx_n = (B.nbx + PAIR_TX - 1) / PAIR_TX, ty_n = (B.nby + PAIR_TY - 1) / PAIR_TY;
    tile_ok = tile < tx_n * ty_n;
    li[0] = (tile % tx_n) * PAIR_TX + 2 * (vl % (PAIR_TX / 2));
    li[1] = (tile / tx_n) * PAIR_TY + vl / (PAIR_TX / 2);
    li[2] = 0;
    a_ok = tile_ok && li[0] < B.nbx && li[1] < B.nby;
    b_ok = a_ok && li[0] + 1 < B.nbx;
}

// bp_step_body for 2D: each lane two x-adjacent voxels (bp_voxel_pair_view_2d), the
// same per-voxel update for both.
template <bool SUB, int SPLIT>
__device__ __forceinline__ void bp_step_body_2d(const DevGeom& G, const int32_t* __restrict__ S_,
                                                const PairWork* __restrict__ work, SchedLayout L,
                                                const float* __restrict__ src, float* __restrict__ ghat,
                                                float* __restrict__ gsum, float* __restrict__ x,
                                                float* __restrict__ xT, const float* __restrict__ mu_ptr,
                                                long long n_vox, int bx, int by, float (&part)[SPLIT][2][BP_VOX])
{
    const int b = by;
    const int j = S_[L.off_blocks() + b];
    const BlockInfo B = G.blocks[j];
    int nb[3];
    float h[3], vs[3];
    block_dims(G, B, nb, h, vs);
    const int vl = threadIdx.x % BP_VOX;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / BP_VOX);
    int li[3];
    bool tile_ok, a_ok, b_ok;
    pair_tile_voxels(B, bx, vl, li, tile_ok, a_ok, b_ok);
    if (!tile_ok) return;  // uniform over the workgroup
    const int64_t vox = ((int64_t)(B.y0 + li[1])) * (int64_t)G.nx + (B.x0 + li[0]);
    const int per_view = G.nu;
    const PairWork* wb = work + (int64_t)b * L.maxv;
    float dga = 0.0f, dgb = 0.0f;
    // the lanes that update the voxels load g and x before the views, so the loads are
    // in flight while the sums are gathered
    const bool upd = grp == 0 && a_ok;
    float gsa = 0.0f, gsb = 0.0f, xva = 0.0f, xvb = 0.0f;
    if (upd) {
        gsa = gsum[vox];
        xva = x[vox];
        if (b_ok) {
            gsb = gsum[vox + 1];
            xvb = x[vox + 1];
        }
    }
    for (int ri = 0; ri < L.R; ++ri) {
        const int a0 = S_[L.off_gstart() + ri], a1 = S_[L.off_gstart() + ri + 1];
        float acc_a = 0.0f, acc_b = 0.0f;
        // this row block's old memories, loaded the same way
        float goa = 0.0f, gob = 0.0f;
        float* gp = nullptr;
        if (!SUB && upd) {
            gp = ghat + (int64_t)S_[L.off_rows() + ri] * n_vox + vox;
            goa = gp[0];
            if (b_ok) gob = gp[1];
        }
        if (a_ok) {
            for (int a = a0 + grp; a < a1; a += SPLIT) {
                const PairWork W = wb[a];
                if (W.k1 <= W.k0) continue;
                if (SUB)
                    bp_voxel_pair_view_2d<false>(G, W.view, W.c, W.s, W, li, b_ok, h, vs, W.k0, W.k1, src + W.zbase,
                                                 acc_a, acc_b);
                else
                    bp_voxel_pair_view_2d<true>(G, W.view, W.c, W.s, W, li, b_ok, h, vs, W.k0, W.k1,
                                                src + (int64_t)a * per_view * 4, acc_a, acc_b);
            }
        }
        part[grp][0][vl] = acc_a;
        part[grp][1][vl] = acc_b;
        __syncthreads();
        if (grp == 0 && a_ok) {
            float sa = part[0][0][vl], sb = part[0][1][vl];
#pragma unroll
            for (int q = 1; q < SPLIT; ++q) {
                sa += part[q][0][vl];
                sb += part[q][1][vl];
            }
            if (SUB) {
                dga += 2.0f * sa;
                dgb += 2.0f * sb;
            } else {
                const float ga = 2.0f * sa;
                dga += ga - goa;
                gp[0] = ga;
                if (b_ok) {
                    const float gb = 2.0f * sb;
                    dgb += gb - gob;
                    gp[1] = gb;
                }
            }
        }
        __syncthreads();
    }
    if (upd) {
        const float mu = *mu_ptr;
        const float gva = gsa + dga;
        gsum[vox] = gva;
        const float xa = fmaf(mu, gva, xva);
        x[vox] = xa;
        // the copy of x stored y fastest (a wave's lanes cover 8 rows of y per x)
        const int64_t tvox = (int64_t)(B.x0 + li[0]) * G.ny + (B.y0 + li[1]);
        if (xT) xT[tvox] = xa;
        if (b_ok) {
            const float gvb = gsb + dgb;
            gsum[vox + 1] = gvb;
            const float xb = fmaf(mu, gvb, xvb);
            x[vox + 1] = xb;
            if (xT) xT[tvox + G.ny] = xb;
        }
    }
}

// ------------------------------------------------------------ 3D back projection: voxel columns

// Each thread owns one voxel column (x, y) of a workgroup tile of BP3_TX x BP3_TY columns
// and up to BP3_CZ voxels in z. Per view, the rays that can cross the column are the
// pixels of the column's shadow: detector columns k from the projections of its four
// xy corners, and per k the rows l from the z range of the column segment the ray's
// xy line cuts out (the xy slab interval [te, tx], which is shared by every row of
// that detector column because all rays of one detector column lie in one vertical
// plane through the source). Each such row crosses one voxel of the column, or two
// (rarely more): the pieces of [te, tx] between the z planes, with the plane crossings
// computed by the forward walk's plane formula. The views' residuals, scaled by the
// ray lengths |d|, are staged in LDS per round of BP3_VC views over the rectangle the
// workgroup tile projects to; a thread adds its pieces into its own LDS accumulators
// (one per voxel of its column), so every voxel's sum is gathered by one thread in a
// fixed order: views ascending, detector columns ascending, rows ascending.
constexpr int BP3_TX = 16, BP3_TY = 16, BP3_WG = BP3_TX * BP3_TY;
constexpr int BP3_CZ = 16;
constexpr int BP3_VC = 5;
constexpr float BP3_EPS = 1e-3f;       // candidate margin of a column's shadow (pixels)
constexpr float BP3_RECT_EPS = 4e-3f;  // margin of the staged rectangle (pixels), wider than BP3_EPS

// plane_pos of a plane index held exactly in a float (the same FMA on the same value).
__device__ __forceinline__ float plane_pos_f(float i, float v, float h) { return fmaf(i, v, -h); }

// One view of a staging round (LDS, written by the first wave).
struct Bp3View {
    int k0, k1, l0, l1;  // pixel rectangle of the workgroup tile in this view, inside the pair's range
    int staged;          // the rectangle's rays are in LDS (else lanes read global memory)
    int a;               // view slot
    int pad0, pad1;
};

// Dynamic LDS layout: accumulators [BP3_CZ + 2][BP3_WG] (voxel iz of a thread's column in
// row iz + 1; rows 0 and nzc + 1 absorb the pieces of rays above or below the column, so
// every add is unconditional), then per view of a round the
// Bp3View, the detector-column records {1/a, 1/b, p_x, p_y} [kmax], the row records
// {p_z, 1/v} [lmax] and the tile of r |d| [lmax][kmax].
__host__ __device__ inline size_t bp3_lds_bytes(const DevGeom& G)
{
    const size_t km = (size_t)G.bp3_kmax, lm = (size_t)G.bp3_lmax;
    return (size_t)(BP3_CZ + 2) * BP3_WG * sizeof(float) +
           (size_t)BP3_VC * (sizeof(Bp3View) + km * sizeof(float4) + lm * sizeof(float2) + km * lm * sizeof(float));
}

// Workgroup tiles per block for the largest block.
__host__ __device__ inline int bp3_tiles(const DevGeom& G)
{
    const int mbx = (G.nx + G.bx - 1) / G.bx, mby = (G.ny + G.by - 1) / G.by, mbz = (G.nz + G.bz - 1) / G.bz;
    return ((mbx + BP3_TX - 1) / BP3_TX) * ((mby + BP3_TY - 1) / BP3_TY) * ((mbz + BP3_CZ - 1) / BP3_CZ);
}

// Views of a solver iteration: work records of the selected pairs; the source is the
// selected rows' residuals (slot a at a * per_view), or with the sub-detector memory
// the residual changes in each pair's z layout.
struct Bp3StepViews {
    const PairWork* wb;
    const float* src;
    int per_view, nu;
    bool sub;
    __device__ __forceinline__ bool get(int a, PairWork& W, const float*& p, int& stride) const
    {
        W = wb[a];
        if (W.k1 <= W.k0 || W.l1 <= W.l0) return false;
        if (sub) {
            p = src + W.zbase;
            stride = W.zw;
        } else {
            p = src + (int64_t)a * per_view;
            stride = nu;
        }
        return true;
    }
};

// Views of a standalone back projection: a view list, whole footprints of block j.
struct Bp3FullViews {
    const PairInfo* pairs;
    const float2* cs;
    const int32_t* views;
    const float* y;
    int j, n_blocks, per_view, nu;
    __device__ __forceinline__ bool get(int a, PairWork& W, const float*& p, int& stride) const
    {
        const int v = views[a];
        const PairInfo P = pairs[(int64_t)v * n_blocks + j];
        if (P.u1 <= P.u0 || P.v1 <= P.v0) return false;
        const float2 sc = cs[v];
        W.k0 = P.u0;
        W.k1 = P.u1;
        W.l0 = P.v0;
        W.l1 = P.v1;
        W.zbase = 0;
        W.zw = 0;
        W.view = v;
        W.au = P.au;
        W.bu = P.bu;
        W.av = P.av;
        W.bv = P.bv;
        W.kc = P.kc;
        W.lc = P.lc;
        W.cu = P.cu;
        W.depth = P.depth;
        W.cz = P.cz;
        W.c = sc.x;
        W.s = sc.y;
        W.pad = 0;
        p = y + (int64_t)a * per_view;
        stride = nu;
        return true;
    }
};

// Detector-column record of ray column k: reciprocal direction (x, y) and the ray's
// block-local xy point (as make_ray).
__device__ __forceinline__ float4 bp3_kcol(const DevGeom& G, const PairWork& W, int k)
{
    const float lu = fmaf((float)(k - W.kc), W.au, W.bu);
    const float4 T = G.raydir[(int64_t)W.view * G.nu + k];
    return make_float4(T.x, T.y, -lu * W.s, lu * W.c);
}

// Row record of ray row l: block-local z of its point and reciprocal z direction (a
// horizontal row's infinite reciprocal replaced by 1e30, so that a cut never computes
// 0 * inf; its cuts then clamp to the segment's ends).
__device__ __forceinline__ float2 bp3_row(const DevGeom& G, const PairWork& W, int l)
{
    const float iv = G.rayv[l].x;
    return make_float2(fmaf((float)(l - W.lc), W.av, W.bv), axis_fixed(iv) ? 1e30f : iv);
}

// Row record of the one-cut form (geometries where no chord through a voxel column
// meets two z planes): {plane_pos(zc0 + up - 1) - z_l, 1/v_l}, up = 1 when the ray
// rises with t. The plane between a ray's entry voxel e (column-local) and its exit
// voxel is then at block-local height plane_pos(zc0 + e + up), and
// (e + 1) v_z + x is that height minus z_l; e + 1 is the entry voxel's accumulator row.
__device__ __forceinline__ float2 bp3_row_cut(const DevGeom& G, const PairWork& W, int l, int zc0, float hz)
{
    const float2 R = bp3_row(G, W, l);
    const int up = R.y > 0.0f ? 1 : 0;
    return make_float2(plane_pos(zc0 + up - 1, G.vz, hz) - R.x, R.y);
}

// r |d| of ray (k, l).
__device__ __forceinline__ float bp3_rlen(const DevGeom& G, const PairWork& W, const float* p, int stride, int k, int l)
{
    const float T2 = G.raydir[(int64_t)W.view * G.nu + k].z;
    return p[(int64_t)l * stride + k] * __builtin_amdgcn_sqrtf(T2 + G.rayv[l].y);
}

// The column's contributions from one view: adds sum a_ij r_i of every ray of the view
// to the thread's accumulators acc[(iz + 1) * BP3_WG] (iz < nzc). STAGED: the rectangle
// [R.k0, R.k1) x [R.l0, R.l1) is in LDS (kc, rw, tile); else from global memory.
template <bool STAGED, bool STEEP>
__device__ __forceinline__ void bp3_column_view(const DevGeom& G, const PairWork& W, const Bp3View& R,
                                                const float* p, int stride, const float4* kc, const float2* rw,
                                                const float* tile, int cx, int cy, int zc0, int nzc,
                                                const float (&h)[3], float* acc)
{
    const float vx = G.vx, vy = G.vy, vz = G.vz;
    const float X0 = plane_pos(cx, vx, h[0]), X1 = plane_pos(cx + 1, vx, h[0]);
    const float Y0 = plane_pos(cy, vy, h[1]), Y1 = plane_pos(cy + 1, vy, h[1]);
    // detector columns of the column's shadow: projections of its four xy corners
    const float c = W.c, s = W.s;
    const float ku = 0.5f * (float)(G.nu - 1), lv = 0.5f * (float)(G.nv - 1);
    const float inv_du = __builtin_amdgcn_rcpf(G.du);
    float kmin = INFINITY, kmax = -INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float X = (q & 1) ? X1 : X0, Y = (q & 2) ? Y1 : Y0;
        const float w = fmaf(Y, c, -(X * s)) + W.cu;
        const float dep = W.depth - fmaf(X, c, Y * s);
        const float kk = fmaf(G.sdd * w * __builtin_amdgcn_rcpf(dep), inv_du, ku);
        kmin = fminf(kmin, kk);
        kmax = fmaxf(kmax, kk);
    }
    const int klo = max(R.k0, (int)ceilf(fminf(fmaxf(kmin - BP3_EPS, (float)R.k0), (float)R.k1)));
    const int khi = min(R.k1 - 1, (int)floorf(fmaxf(fminf(kmax + BP3_EPS, (float)R.k1), (float)R.k0 - 1.0f)));
    // z planes of the column: block-local and absolute
    const float zb = plane_pos(zc0, vz, h[2]);
    const float zt = plane_pos(zc0 + nzc, vz, h[2]);
    const float zb_abs = zb + W.cz, zt_abs = zt + W.cz;
    const float A = W.depth * __builtin_amdgcn_rcpf(G.sdd);  // depth of the ray parameter origin / sdd
    const float inv_vz = __builtin_amdgcn_rcpf(vz);
    const float dv = G.dv;
    const int w_tile = R.k1 - R.k0;
    const int tid = threadIdx.x;
    const float nzf = (float)nzc, zcf = (float)zc0;
    for (int k = klo; k <= khi; ++k) {
        float4 K;
        if constexpr (STAGED)
            K = kc[k - R.k0];
        else
            K = bp3_kcol(G, W, k);
        float te = -INFINITY, tx = INFINITY;
        bool hit = true;
        slab_axis(K.z, K.x, cx, vx, h[0], te, tx, hit);
        slab_axis(K.w, K.y, cy, vy, h[1], te, tx, hit);
        if (!hit || !(te < tx)) continue;
        // rows whose ray meets the column between te and tx: row of an absolute height Z
        // at parameter t is lv + Z / ((A + t) dv)
        const float rfe = __builtin_amdgcn_rcpf((A + te) * dv), rfx = __builtin_amdgcn_rcpf((A + tx) * dv);
        const float lmin = fminf(zb_abs * rfe, zb_abs * rfx) + lv;
        const float lmax = fmaxf(zt_abs * rfe, zt_abs * rfx) + lv;
        const int llo = max(R.l0, (int)ceilf(fminf(fmaxf(lmin - BP3_EPS, (float)R.l0), (float)R.l1)));
        const int lhi = min(R.l1 - 1, (int)floorf(fmaxf(fminf(lmax + BP3_EPS, (float)R.l1), (float)R.l0 - 1.0f)));
        // the height of row l's ray at te and tx, in voxels above the column's bottom
        // plane, is affine in l (used only to pick the voxels; the cut points below
        // use the exact plane formula and are clamped to [te, tx])
        const float se = fmaf(te, dv, W.av) * inv_vz, sx = fmaf(tx, dv, W.av) * inv_vz;
        const float o0 = fmaf(-(float)W.lc, W.av, W.bv) - zb;
        float ue = fmaf((float)llo, se, fmaf(-te * lv, dv, o0) * inv_vz);
        float ux = fmaf((float)llo, sx, fmaf(-tx * lv, dv, o0) * inv_vz);
        const float2* rwp = nullptr;
        const float* tp = nullptr;
        if constexpr (STAGED) {
            rwp = rw + (llo - R.l0);
            tp = tile + (llo - R.l0) * w_tile + (k - R.k0);
        }
        if constexpr (STAGED && !STEEP) {
            // One cut per row, at the plane beyond the entry voxel in the ray's z
            // direction (rows staged by bp3_row_cut). Heights are kept one voxel up, so
            // the clamped truncation is the accumulator row (voxel + 1; rows 0 and
            // nzc + 1 are the spares). When entry and exit rows coincide the cut clamps
            // to te or tx and the two pieces add to the whole chord: the exit piece is
            // added first and the entry write, made last, carries both.
            ue += 1.0f;
            ux += 1.0f;
            const float top = nzf + 1.0f;
            float* const accp = acc + tid;
            for (int l = llo; l <= lhi; ++l) {
                const float2 Rw = *rwp++;
                const float rl = *tp;
                tp += w_tile;
                const float fe = truncf(__builtin_amdgcn_fmed3f(ue, 0.0f, top));
                const int re = (int)fe;
                const int rx = (int)__builtin_amdgcn_fmed3f(ux, 0.0f, top);
                ue += se;
                ux += sx;
                const float ts = __builtin_amdgcn_fmed3f(fmaf(fe, vz, Rw.x) * Rw.y, te, tx);
                float* p0 = accp + re * BP3_WG;
                float* p1 = accp + rx * BP3_WG;
                const float v0 = *p0, v1 = *p1;
                const float n1 = fmaf(tx - ts, rl, v1);
                const float n0 = fmaf(ts - te, rl, re == rx ? n1 : v0);
                *p1 = n1;
                *p0 = n0;
            }
            continue;
        }
        for (int l = llo; l <= lhi; ++l) {
            float2 Rw;
            float rl;
            if constexpr (STAGED) {
                Rw = *rwp++;
                rl = *tp;
                tp += w_tile;
            } else {
                Rw = bp3_row(G, W, l);
                rl = bp3_rlen(G, W, p, stride, k, l);
            }
            // voxels (column-local, -1 and nzc = outside) holding the ray at te and tx
            const float fe = floorf(__builtin_amdgcn_fmed3f(ue, -1.0f, nzf));
            const float fx = floorf(__builtin_amdgcn_fmed3f(ux, -1.0f, nzf));
            ue += se;
            ux += sx;
            // one cut, at the plane between the two voxels (the upper one's bottom); on
            // one voxel the whole chord is its own and the second (zero) piece goes to
            // the spare row 0. Plain LDS read-add-write (each thread owns its
            // accumulators; LDS atomics serialise lanes): both reads, then the writes in
            // program order, the two addresses distinct.
            const bool one = fe == fx;
            const float zcut = plane_pos_f(zcf + fmaxf(fe, fx), vz, h[2]);
            const float ts = one ? tx : __builtin_amdgcn_fmed3f((zcut - Rw.x) * Rw.y, te, tx);
            float* p0 = acc + (int)fmaf(fe, (float)BP3_WG, (float)(BP3_WG + tid));
            float* p1 = acc + (one ? tid : (int)fmaf(fx, (float)BP3_WG, (float)(BP3_WG + tid)));
            const float v0 = *p0, v1 = *p1;
            *p0 = fmaf(ts - te, rl, v0);
            float tl = ts;
            if constexpr (STEEP) {
                const int ie = (int)fe, ix = (int)fx, d = ix - ie;
                if (d > 1 || d < -1) {
                    // more than one plane inside [te, tx]: the voxels between (the cut
                    // above is then the first one, at the plane next to voxel ie)
                    const int st = d > 0 ? 1 : -1;
                    tl = __builtin_amdgcn_fmed3f(plane_t(zc0 + ie + (st > 0 ? 1 : 0), vz, h[2], Rw.x, Rw.y), te, tx);
                    *p0 = fmaf(tl - te, rl, v0);
                    for (int i = ie + st; i != ix; i += st) {
                        const float tn =
                            __builtin_amdgcn_fmed3f(plane_t(zc0 + i + (st > 0 ? 1 : 0), vz, h[2], Rw.x, Rw.y), tl, tx);
                        float* pm = acc + (i + 1) * BP3_WG + tid;
                        *pm = fmaf(tn - tl, rl, *pm);
                        tl = tn;
                    }
                }
            }
            *p1 = fmaf(tx - tl, rl, v1);
        }
    }
}

// Back projection of views [a0, a1) of `views` into the columns of one workgroup tile
// (block-local columns (tx0 + threadIdx.x % BP3_TX, ty0 + threadIdx.x / BP3_TX), z voxels
// [zc0, zc0 + nzc)): acc[(iz + 1) * BP3_WG + threadIdx.x] += sum over the views' rays of a_ij r_i.
// Every thread of the workgroup must call it (barriers).
template <class Views>
__device__ __forceinline__ void bp3_accumulate(const DevGeom& G, const BlockInfo& B, const Views& views, int a0,
                                               int a1, int tx0, int ty0, int zc0, int nzc, float* lds)
{
    float* acc = lds;
    Bp3View* rec = reinterpret_cast<Bp3View*>(acc + (BP3_CZ + 2) * BP3_WG);
    const int km = G.bp3_kmax, lm = G.bp3_lmax;
    float4* kc_all = reinterpret_cast<float4*>(rec + BP3_VC);
    float2* rw_all = reinterpret_cast<float2*>(kc_all + BP3_VC * km);
    float* tile_all = reinterpret_cast<float*>(rw_all + BP3_VC * lm);
    float h[3];
    h[0] = B.hx;
    h[1] = B.hy;
    h[2] = B.hz;
    const int cx = tx0 + (int)threadIdx.x % BP3_TX, cy = ty0 + (int)threadIdx.x / BP3_TX;
    const bool col_ok = cx < B.nbx && cy < B.nby;
    const int tx1 = min(tx0 + BP3_TX, B.nbx), ty1 = min(ty0 + BP3_TY, B.nby);
    // workgroups start with rounds of 5, 4, 3 or 2 views by their id, so that workgroups
    // sharing a CU stage at different times (the views and their order are the same)
    const int phase = (int)((blockIdx.y * gridDim.x + blockIdx.x) & 3);
    for (int ab = a0, nvw = min(BP3_VC - phase, a1 - a0); ab < a1; ab += nvw, nvw = min(BP3_VC, a1 - ab)) {
        __syncthreads();  // the previous round's readers are done
        if (threadIdx.x < 64) {
            // lanes 8q .. 8q+7: the eight corners of the tile in view slot ab + q
            const int q = (int)threadIdx.x >> 3, corner = (int)threadIdx.x & 7;
            PairWork W;
            const float* p;
            int stride;
            const bool ok = q < nvw && views.get(ab + q, W, p, stride);
            float kk = 0.0f, ll = 0.0f;
            if (ok) {
                const float X = plane_pos((corner & 1) ? tx1 : tx0, G.vx, h[0]);
                const float Y = plane_pos((corner & 2) ? ty1 : ty0, G.vy, h[1]);
                const float Z = plane_pos((corner & 4) ? zc0 + nzc : zc0, G.vz, h[2]) + W.cz;
                const float w = fmaf(Y, W.c, -(X * W.s)) + W.cu;
                const float rdep = __builtin_amdgcn_rcpf(W.depth - fmaf(X, W.c, Y * W.s));
                kk = fmaf(G.sdd * w * rdep, __builtin_amdgcn_rcpf(G.du), 0.5f * (float)(G.nu - 1));
                ll = fmaf(G.sdd * Z * rdep, __builtin_amdgcn_rcpf(G.dv), 0.5f * (float)(G.nv - 1));
            }
            float kmin = kk, kmax = kk, lmin = ll, lmax = ll;
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                kmin = fminf(kmin, __shfl_xor(kmin, o, 64));
                kmax = fmaxf(kmax, __shfl_xor(kmax, o, 64));
                lmin = fminf(lmin, __shfl_xor(lmin, o, 64));
                lmax = fmaxf(lmax, __shfl_xor(lmax, o, 64));
            }
            if (corner == 0 && q < BP3_VC) {
                Bp3View r;
                r.a = ab + q;
                r.pad0 = r.pad1 = 0;
                if (ok) {
                    r.k0 = max(W.k0, (int)ceilf(fminf(fmaxf(kmin - BP3_RECT_EPS, (float)W.k0), (float)W.k1)));
                    r.k1 = min(W.k1, (int)floorf(fmaxf(fminf(kmax + BP3_RECT_EPS, (float)W.k1), (float)W.k0 - 1.0f)) + 1);
                    r.l0 = max(W.l0, (int)ceilf(fminf(fmaxf(lmin - BP3_RECT_EPS, (float)W.l0), (float)W.l1)));
                    r.l1 = min(W.l1, (int)floorf(fmaxf(fminf(lmax + BP3_RECT_EPS, (float)W.l1), (float)W.l0 - 1.0f)) + 1);
                    if (r.k1 <= r.k0 || r.l1 <= r.l0) r.k0 = r.k1 = r.l0 = r.l1 = 0;
                } else {
                    r.k0 = r.k1 = r.l0 = r.l1 = 0;
                }
                r.staged = (r.k1 - r.k0) <= km && (r.l1 - r.l0) <= lm;
                rec[q] = r;
            }
        }
        __syncthreads();
        // stage the rectangles: column records, row records, r |d|
        for (int q = 0; q < nvw; ++q) {
            const Bp3View r = rec[q];
            if (!r.staged || r.k1 <= r.k0) continue;  // uniform
            PairWork W;
            const float* p;
            int stride;
            views.get(r.a, W, p, stride);
            const int wt = r.k1 - r.k0, ht = r.l1 - r.l0;
            float4* kc = kc_all + q * km;
            float2* rw = rw_all + q * lm;
            float* tile = tile_all + q * km * lm;
            for (int e = threadIdx.x; e < wt + ht; e += BP3_WG) {
                if (e < wt)
                    kc[e] = bp3_kcol(G, W, r.k0 + e);
                else
                    rw[e - wt] = G.bp3_steep ? bp3_row(G, W, r.l0 + (e - wt))
                                             : bp3_row_cut(G, W, r.l0 + (e - wt), zc0, h[2]);
            }
            for (int e = threadIdx.x; e < wt * ht; e += BP3_WG) {
                const int l = e / wt, k = e - l * wt;
                tile[e] = bp3_rlen(G, W, p, stride, r.k0 + k, r.l0 + l);
            }
        }
        __syncthreads();
        if (!col_ok) continue;
        for (int q = 0; q < nvw; ++q) {
            const Bp3View r = rec[q];
            if (r.k1 <= r.k0) continue;  // uniform
            PairWork W;
            const float* p;
            int stride;
            views.get(r.a, W, p, stride);
            if (r.staged) {
                if (G.bp3_steep)
                    bp3_column_view<true, true>(G, W, r, p, stride, kc_all + q * km, rw_all + q * lm,
                                                tile_all + q * km * lm, cx, cy, zc0, nzc, h, acc);
                else
                    bp3_column_view<true, false>(G, W, r, p, stride, kc_all + q * km, rw_all + q * lm,
                                                 tile_all + q * km * lm, cx, cy, zc0, nzc, h, acc);
            } else {
                bp3_column_view<false, true>(G, W, r, p, stride, nullptr, nullptr, nullptr, cx, cy, zc0, nzc, h, acc);
            }
        }
    }
    __syncthreads();
}

// Workgroup tile `tile` of block B: first column (tx0, ty0) and z range [zc0, zc0 + nzc);
// false when the block has fewer tiles (uniform).
__device__ __forceinline__ bool bp3_tile(const BlockInfo& B, int tile, int& tx0, int& ty0, int& zc0, int& nzc)
{
    const int ntx = (B.nbx + BP3_TX - 1) / BP3_TX, nty = (B.nby + BP3_TY - 1) / BP3_TY;
    const int ntz = (B.nbz + BP3_CZ - 1) / BP3_CZ;
    if (tile >= ntx * nty * ntz) return false;
    tx0 = (tile % ntx) * BP3_TX;
    ty0 = ((tile / ntx) % nty) * BP3_TY;
    zc0 = (tile / (ntx * nty)) * BP3_CZ;
    nzc = min(BP3_CZ, B.nbz - zc0);
    return true;
}

// Solver step for 3D blocks (bp_step_body's contract): per selected row block the
// column sums give g_hat^i_new = 2 (A_rows^J)^T r, then g and x as in the 2D form.
template <bool SUB>
__device__ __forceinline__ void bp3_step_body(const DevGeom& G, const int32_t* __restrict__ S_,
                                              const PairWork* __restrict__ work, SchedLayout L,
                                              const float* __restrict__ src, float* __restrict__ ghat,
                                              float* __restrict__ gsum, float* __restrict__ x,
                                              float* __restrict__ xT, const float* __restrict__ mu_ptr,
                                              long long n_vox, int bx, int by, float* lds)
{
    const int b = by;
    const int j = S_[L.off_blocks() + b];
    const BlockInfo B = G.blocks[j];
    int tx0, ty0, zc0, nzc;
    if (!bp3_tile(B, bx, tx0, ty0, zc0, nzc)) return;  // uniform over the workgroup
    float* acc = lds;
    const int cx = tx0 + (int)threadIdx.x % BP3_TX, cy = ty0 + (int)threadIdx.x / BP3_TX;
    const bool col_ok = cx < B.nbx && cy < B.nby;
#pragma unroll
    for (int iz = 0; iz < BP3_CZ + 2; ++iz) acc[iz * BP3_WG + threadIdx.x] = 0.0f;
    const Bp3StepViews views{work + (int64_t)b * L.maxv, src, G.nu * G.nv, G.nu, SUB};
    const int64_t plane = (int64_t)G.nx * G.ny;
    const int64_t vox0 = ((int64_t)(B.z0 + zc0) * G.ny + (B.y0 + cy)) * (int64_t)G.nx + (B.x0 + cx);
    float dg[BP3_CZ];
#pragma unroll
    for (int iz = 0; iz < BP3_CZ; ++iz) dg[iz] = 0.0f;
    if (!SUB && L.R == 1) {
        // one row block: its old memories are loaded into dg before the accumulation, so
        // they arrive with the first staging loads instead of after the last view; then
        // dg = g_hat_new - g_hat_old, the same value as below
        const int i = S_[L.off_rows()];
        if (col_ok) {
#pragma unroll
            for (int iz = 0; iz < BP3_CZ; ++iz)
                if (iz < nzc) dg[iz] = ghat[(int64_t)i * n_vox + vox0 + iz * plane];
        }
        bp3_accumulate(G, B, views, S_[L.off_gstart()], S_[L.off_gstart() + 1], tx0, ty0, zc0, nzc, lds);
        if (col_ok) {
#pragma unroll
            for (int iz = 0; iz < BP3_CZ; ++iz) {
                if (iz < nzc) {
                    float* ap = acc + (iz + 1) * BP3_WG + threadIdx.x;
                    const float gnew = 2.0f * *ap;
                    *ap = 0.0f;
                    dg[iz] = gnew - dg[iz];
                    ghat[(int64_t)i * n_vox + vox0 + iz * plane] = gnew;
                }
            }
        }
    } else {
        for (int ri = 0; ri < L.R; ++ri) {
            const int a0 = S_[L.off_gstart() + ri], a1 = S_[L.off_gstart() + ri + 1];
            bp3_accumulate(G, B, views, a0, a1, tx0, ty0, zc0, nzc, lds);
            if (col_ok) {
                const int i = S_[L.off_rows() + ri];
#pragma unroll
                for (int iz = 0; iz < BP3_CZ; ++iz) {
                    if (iz < nzc) {
                        float* ap = acc + (iz + 1) * BP3_WG + threadIdx.x;
                        const float gnew = 2.0f * *ap;
                        *ap = 0.0f;
                        if (SUB) {
                            dg[iz] += gnew;
                        } else {
                            float* gp = ghat + (int64_t)i * n_vox + vox0 + iz * plane;
                            dg[iz] += gnew - *gp;
                            *gp = gnew;
                        }
                    }
                }
            }
        }
    }
    if (col_ok) {
        const float mu = *mu_ptr;
#pragma unroll
        for (int iz = 0; iz < BP3_CZ; ++iz) {
            if (iz < nzc) {
                const int64_t vox = vox0 + iz * plane;
                const float gv = gsum[vox] + dg[iz];
                gsum[vox] = gv;
                const float xv = fmaf(mu, gv, x[vox]);
                x[vox] = xv;
                // staged for the copy of x stored y fastest (each thread's own slots of
                // the accumulator rows, which it no longer reads)
                if (xT) acc[iz * BP3_WG + threadIdx.x] = xv;
            }
        }
    }
    if (xT) {  // uniform
        // the tile's new values into xT, threads over (x, y) with y fastest
        __syncthreads();
        const int ty = (int)threadIdx.x % BP3_TY, tx = (int)threadIdx.x / BP3_TY;
        if (tx0 + tx < B.nbx && ty0 + ty < B.nby) {
            const int64_t t0 =
                ((int64_t)(B.z0 + zc0) * G.nx + (B.x0 + tx0 + tx)) * (int64_t)G.ny + (B.y0 + ty0 + ty);
#pragma unroll
            for (int iz = 0; iz < BP3_CZ; ++iz)
                if (iz < nzc) xT[t0 + iz * plane] = acc[iz * BP3_WG + ty * BP3_TX + tx];
        }
    }
}

// Workgroup size of the back projectors: 2D `split` waves of pair tiles; 3D one thread
// per voxel column of a 16 x 16 column tile.
__host__ __device__ constexpr int bp_wg(int dim, int split = BP_SPLIT_2D)
{
    return dim == 3 ? BP3_WG : BP_VOX * split;
}

template <int DIM, bool SUB, int SPLIT = BP_SPLIT_2D>
__global__ __launch_bounds__(bp_wg(DIM, SPLIT)) void k_bp_step(DevGeom G, const int32_t* __restrict__ S_,
                                                              const PairWork* __restrict__ work, SchedLayout L,
                                                              const float* __restrict__ src,
                                                              float* __restrict__ ghat, float* __restrict__ gsum,
                                                              float* __restrict__ x, float* __restrict__ xT,
                                                              const float* __restrict__ mu, long long n_vox)
{
    int bx, by;
    xcd_grid2(bx, by);
    if constexpr (DIM == 2) {
        __shared__ float part[SPLIT][2][BP_VOX];
        bp_step_body_2d<SUB, SPLIT>(G, S_, work, L, src, ghat, gsum, x, xT, mu, n_vox, bx, by, part);
    } else {
        extern __shared__ float bp3_lds[];
        bp3_step_body<SUB>(G, S_, work, L, src, ghat, gsum, x, xT, mu, n_vox, bx, by, bp3_lds);
    }
}

// Sub-detector gradient memory: one workgroup per (view slot, block slot) pair. Over the
// pair's pixel range, d = r - rho (the change of each ray's residual since the pair's
// view, sub-detector and block last ran) and rho = r, both in the pair's z layout. A
// (view, block) pair occurs at most once per iteration, so no two workgroups share a
// pixel.
__global__ __launch_bounds__(WG) void k_subdet_delta(DevGeom G, const int32_t* __restrict__ S_,
                                                     const PairWork* __restrict__ work, SchedLayout L,
                                                     const float* __restrict__ r_sel, float* __restrict__ rho,
                                                     float* __restrict__ delta)
{
    const int a = blockIdx.x, b = blockIdx.y;
    if (a >= S_[0]) return;
    const PairWork W = work[(int64_t)b * L.maxv + a];
    const int w = W.k1 - W.k0, hgt = W.l1 - W.l0;
    if (w <= 0 || hgt <= 0) return;
    const int64_t row = (int64_t)a * G.nu * G.nv;
    const int n = w * hgt;
    for (int t = threadIdx.x; t < n; t += WG) {
        const int k = W.k0 + t % w, l = W.l0 + t / w;
        const int64_t zi = W.zbase + (int64_t)l * W.zw + k;
        const int64_t q = row + (int64_t)l * G.nu + k;
        const float rr = G.dim == 2 ? reinterpret_cast<const float4*>(r_sel)[q].w : r_sel[q];
        delta[zi] = rr - rho[zi];
        rho[zi] = rr;
    }
}

// ------------------------------------------------------------ batched solves

// Many solves in one launch per phase: workgroup id -> (entry, local workgroup) by a
// binary search over each entry's first workgroup; the entry's own body then runs
// exactly as in the single-solve kernels, so a solve's arithmetic does not depend on
// the batch it runs in.
__device__ __forceinline__ int find_entry(const BatchEntry* E, int n, int phase, int id)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (E[mid].base[phase] <= id) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// TPB: FP_LDS_WG for the LDS-staged entries' launch classes, WG for the global-memory
// class (whose per-entry grid counts WG / 64 waves per workgroup); a class never mixes
// the two (their LDS sizes differ).
template <int DIM, int TPB>
__global__ __launch_bounds__(TPB) void k_fp_batch(const BatchArgs A)
{
    extern __shared__ float xs[];
    __shared__ FpLds sh;
    const int id = A.id0 + xcd_local((int)blockIdx.x, (int)gridDim.x);
    const int e = __builtin_amdgcn_readfirstlane(find_entry(A.e, A.n, 0, id));
    const BatchEntry& B = A.e[e];
    const int local = id - B.base[0];
    const int32_t* S_ = B.sched + (int64_t)A.it * B.L.stride;
    const PairWork* W = B.work + (int64_t)A.it * B.L.maxv * B.L.B;
    if (TPB == FP_LDS_WG) {
        if (B.fp_lds)
            fp_lds_body<DIM, TPB>(B.G, W, B.L, S_ + B.L.off_blocks(), B.x, B.z, B.fp_chunk, local % B.gx[0],
                                  local / B.gx[0], xs, sh);
    } else if (!B.fp_lds) {
        const int wave = __builtin_amdgcn_readfirstlane(local * (TPB / 64) + (threadIdx.x >> 6));
        fp_global_body<DIM>(B.G, W, B.L, S_ + B.L.off_blocks(), B.x, B.xT, B.z, wave, threadIdx.x & 63);
    }
}

template <int TPB>
__global__ __launch_bounds__(TPB) void k_resid_batch(const BatchArgs A)
{
    extern __shared__ int4 rc[];
    const int id = xcd_local((int)blockIdx.x, (int)gridDim.x);
    const int e = __builtin_amdgcn_readfirstlane(find_entry(A.e, A.n, 1, id));
    const BatchEntry& B = A.e[e];
    const int local = id - B.base[1];
    const int32_t* S_ = B.sched + (int64_t)A.it * B.L.stride;
    resid_body<TPB>(B.G, S_, B.L, B.y, B.z, B.r_sel, local % B.gx[1], local / B.gx[1], rc);
}

template <int DIM, int SPLIT = BP_SPLIT_2D>
__global__ __launch_bounds__(bp_wg(DIM, SPLIT)) void k_bp_batch(const BatchArgs A)
{
    const int id = A.id0 + xcd_local((int)blockIdx.x, (int)gridDim.x);
    const int e = __builtin_amdgcn_readfirstlane(find_entry(A.e, A.n, 2, id));
    const BatchEntry& B = A.e[e];
    const int local = id - B.base[2];
    const int32_t* S_ = B.sched + (int64_t)A.it * B.L.stride;
    const PairWork* W = B.work + (int64_t)A.it * B.L.maxv * B.L.B;
    if constexpr (DIM == 2) {
        __shared__ float part[SPLIT][2][BP_VOX];
        bp_step_body_2d<false, SPLIT>(B.G, S_, W, B.L, B.r_sel, B.ghat, B.gsum, B.x, B.xT, B.mu, B.n_vox,
                                      local % B.gx[2], local / B.gx[2], part);
    } else {
        extern __shared__ float bp3_lds[];
        bp3_step_body<false>(B.G, S_, W, B.L, B.r_sel, B.ghat, B.gsum, B.x, B.xT, B.mu, B.n_vox, local % B.gx[2],
                             local / B.gx[2], bp3_lds);
    }
}

// ------------------------------------------------------------ standalone projectors

template <int DIM>
__global__ __launch_bounds__(WG) void k_fp_full(DevGeom G, const int32_t* __restrict__ views, int n_sel,
                                                int j0, int j1, const float* __restrict__ x,
                                                float* __restrict__ y, int accumulate)
{
    const int a = blockIdx.y;
    const int per_view = G.nu * G.nv;
    const int ray = blockIdx.x * WG + threadIdx.x;
    if (a >= n_sel || ray >= per_view) return;
    const int v = views[a];
    const int k = ray % G.nu, l = ray / G.nu;
    const float2 cs = G.cs[v];
    const int64_t sy = G.nx, sz = (int64_t)G.nx * G.ny;
    float acc = 0.0f;
    for (int j = j0; j < j1; ++j) {
        const PairInfo P = G.pairs[(int64_t)v * G.N + j];
        if (k >= P.u0 && k < P.u1 && l >= P.v0 && l < P.v1) {
            const BlockInfo B = G.blocks[j];
            const float* xb = x + ((int64_t)B.z0 * G.ny + B.y0) * (int64_t)G.nx + B.x0;
            acc += fp_ray_block<DIM>(G, v, cs.x, cs.y, P, B, k, l, xb, sy, sz);
        }
    }
    float* dst = y + (int64_t)a * per_view + ray;
    *dst = accumulate ? *dst + acc : acc;
}

// Standalone back projection into block j0 + blockIdx.y, 2D: two x-adjacent voxels per
// lane (pair tiles, as the solver's).
__global__ __launch_bounds__(bp_wg(2)) void k_bp_full_2d(DevGeom G, const int32_t* __restrict__ views, int n_sel, int j0,
                                                 const float* __restrict__ y, float* __restrict__ x, float scale,
                                                 int accumulate)
{
    __shared__ float part[BP_SPLIT_2D][2][BP_VOX];
    const int j = j0 + blockIdx.y;
    const BlockInfo B = G.blocks[j];
    int nb[3];
    float h[3], vs[3];
    block_dims(G, B, nb, h, vs);
    const int vl = threadIdx.x % BP_VOX;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / BP_VOX);
    int li[3];
    bool tile_ok, valid, b_ok = false;
    pair_tile_voxels(B, blockIdx.x, vl, li, tile_ok, valid, b_ok);
    if (!tile_ok) return;
    const int per_view = G.nu * G.nv;
    float acc = 0.0f, acc_b = 0.0f;
    if (valid) {
        for (int a = grp; a < n_sel; a += BP_SPLIT_2D) {
            const int v = views[a];
            const PairInfo P = G.pairs[(int64_t)v * G.N + j];
            if (P.u1 <= P.u0 || P.v1 <= P.v0) continue;
            const float2 cs = G.cs[v];
            bp_voxel_pair_view_2d<false>(G, v, cs.x, cs.y, P, li, b_ok, h, vs, P.u0, P.u1, y + (int64_t)a * per_view,
                                         acc, acc_b);
        }
    }
    part[grp][0][vl] = acc;
    part[grp][1][vl] = acc_b;
    __syncthreads();
    if (grp == 0 && valid) {
        float sum = part[0][0][vl], sum_b = part[0][1][vl];
#pragma unroll
        for (int q = 1; q < BP_SPLIT_2D; ++q) {
            sum += part[q][0][vl];
            sum_b += part[q][1][vl];
        }
        const int64_t vox = ((int64_t)(B.y0 + li[1])) * (int64_t)G.nx + (B.x0 + li[0]);
        const float val = scale * sum;
        x[vox] = accumulate ? x[vox] + val : val;
        if (b_ok) {
            const float vb = scale * sum_b;
            x[vox + 1] = accumulate ? x[vox + 1] + vb : vb;
        }
    }
}

// Standalone back projection into block j0 + blockIdx.y, 3D: voxel-column tiles
// (bp3_accumulate) over the whole view list.
__global__ __launch_bounds__(BP3_WG) void k_bp_full_3d(DevGeom G, const int32_t* __restrict__ views, int n_sel, int j0,
                                                const float* __restrict__ y, float* __restrict__ x, float scale,
                                                int accumulate)
{
    extern __shared__ float bp3_lds[];
    const int j = j0 + blockIdx.y;
    const BlockInfo B = G.blocks[j];
    int tx0, ty0, zc0, nzc;
    if (!bp3_tile(B, blockIdx.x, tx0, ty0, zc0, nzc)) return;  // uniform
    float* acc = bp3_lds;
#pragma unroll
    for (int iz = 0; iz < BP3_CZ + 2; ++iz) acc[iz * BP3_WG + threadIdx.x] = 0.0f;
    const Bp3FullViews fv{G.pairs, G.cs, views, y, j, G.N, G.nu * G.nv, G.nu};
    bp3_accumulate(G, B, fv, 0, n_sel, tx0, ty0, zc0, nzc, bp3_lds);
    const int cx = tx0 + (int)threadIdx.x % BP3_TX, cy = ty0 + (int)threadIdx.x / BP3_TX;
    if (cx >= B.nbx || cy >= B.nby) return;
    const int64_t plane = (int64_t)G.nx * G.ny;
    const int64_t vox0 = ((int64_t)(B.z0 + zc0) * G.ny + (B.y0 + cy)) * (int64_t)G.nx + (B.x0 + cx);
#pragma unroll
    for (int iz = 0; iz < BP3_CZ; ++iz) {
        if (iz < nzc) {
            const int64_t vox = vox0 + iz * plane;
            const float val = scale * acc[(iz + 1) * BP3_WG + threadIdx.x];
            x[vox] = accumulate ? x[vox] + val : val;
        }
    }
}

// ------------------------------------------------------------ reductions

__global__ __launch_bounds__(WG) void k_resid_sumsq(DevGeom G, const float* __restrict__ y,
                                                    const float* __restrict__ z, double* __restrict__ partials)
{
    __shared__ double lds[4];
    extern __shared__ int4 rc[];
    int4* grc = rc + G.N;
    long long* zo = reinterpret_cast<long long*>(grc + res_groups(G));
    long long* cand = zo + G.N + threadIdx.x * res_batch(WG);
    const int v = blockIdx.y;
    const int per_view = G.nu * G.nv;
    const int ray = blockIdx.x * WG + threadIdx.x;
    double val = 0.0;
    if (G.cov_off) {
        if (ray < per_view) {
            const float r = resid_ray_idx<16>(G, (int64_t)v * per_view + ray, y, z);
            val = (double)r * (double)r;
        }
    } else {
        stage_rects(G, v, rc, zo, grc);
        if (ray < per_view) {
            const float r = resid_ray<res_batch(WG)>(G, v, ray % G.nu, ray / G.nu, y, z, rc, zo, grc, cand, per_view,
                                                     ray);
            val = (double)r * (double)r;
        }
    }
    const double s = block_sum(val, lds);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(WG) void k_sumsq(const float* __restrict__ a, long long n, double* __restrict__ partials)
{
    __shared__ double lds[4];
    double val = 0.0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) val += (double)a[i] * (double)a[i];
    const double s = block_sum(val, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(WG) void k_sum_partials(const double* __restrict__ p, int n, double* __restrict__ out)
{
    __shared__ double lds[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += WG) v += p[i];
    const double s = block_sum(v, lds);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(WG) void k_sub(const float* __restrict__ b, const float* __restrict__ c,
                                            float* __restrict__ a, long long n)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) a[i] = b[i] - c[i];
}

__global__ __launch_bounds__(WG) void k_add(float* __restrict__ a, const float* __restrict__ b, long long n)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) a[i] += b[i];
}

__global__ __launch_bounds__(WG) void k_dot(const float* __restrict__ a, const float* __restrict__ b, long long n,
                                            double* __restrict__ partials)
{
    __shared__ double lds[4];
    double val = 0.0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) val += (double)a[i] * (double)b[i];
    const double s = block_sum(val, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(WG) void k_fill(float* __restrict__ a, float v, long long n)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) a[i] = v;
}

// ------------------------------------------------------------ TV proximal step (FGP)

// D^T q at voxel (x, y, z) for the backward-difference gradient with zero
// differences across the low boundary: sum_a [q_a(c) (c_a >= 1) - q_a(c + e_a) (c_a + 1 < n_a)].
template <int DIM>
__device__ __forceinline__ float div_adj(const float* __restrict__ q, int64_t nvox, int X, int Y, int Z, int nx,
                                         int ny, int nz)
{
    const int64_t o = ((int64_t)Z * ny + Y) * nx + X;
    float r = 0.0f;
    if (X >= 1) r += q[o];
    if (X + 1 < nx) r -= q[o + 1];
    if (Y >= 1) r += q[nvox + o];
    if (Y + 1 < ny) r -= q[nvox + o + nx];
    if (DIM == 3) {
        if (Z >= 1) r += q[2 * nvox + o];
        if (Z + 1 < nz) r -= q[2 * nvox + o + (int64_t)nx * ny];
    }
    return r;
}

// One FGP iteration fused into one pass. The dual iterates p_k (pc) and p_{k-1} (pp)
// are kept instead of the extrapolated point, which is rebuilt where it is read:
// r = p_k + coef (p_k - p_{k-1}); then u = b - w D^T r and
// p_{k+1} = P_ball(r + step D u), with D the backward differences (zero across the low
// boundary) and P_ball the projection onto the unit ball per voxel. HBM traffic per voxel:
// p_k and p_{k-1} read, b read, p_{k+1} written (40 B in 3D).
//
// A workgroup owns a FGP_TX x FGP_TY column tile and marches up FGP_ZC planes. Per plane
// it builds r of the next plane in LDS over the tile with a one-voxel halo (three
// planes rotate, so a plane's r is built once), then u of the plane over the tile and
// its low halo, then the dual update of its own voxels; u one plane down stays in a
// register. A chunk starts one plane low (u only) unless it starts at z = 0.
constexpr int FGP_TX = 64, FGP_TY = 8, FGP_ZC = 32, FGP_WG = FGP_TX * FGP_TY;
constexpr int FGP_HX = FGP_TX + 2, FGP_HY = FGP_TY + 2;  // r tile with halo, x and y in [-1, T]
constexpr int FGP_UX = FGP_TX + 1, FGP_UY = FGP_TY + 1;  // u tile with low halo, in [-1, T - 1]

template <int DIM>
__global__ __launch_bounds__(FGP_WG) void k_fgp_step(const float* __restrict__ b, const float* __restrict__ pc,
                                                     const float* __restrict__ pp, float* __restrict__ pn, int nx,
                                                     int ny, int nz, const float* __restrict__ wstep, float coef)
{
    __shared__ float rL[3][DIM][FGP_HY * FGP_HX];
    __shared__ float uL[FGP_UY * FGP_UX];
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t plane = (int64_t)nx * ny;
    // tiles x fastest, then y, then z chunks, numbered so that each XCD marches a
    // contiguous run of them together and the halos its tiles share stay in its L2
    const int gx = (nx + FGP_TX - 1) / FGP_TX, gy = (ny + FGP_TY - 1) / FGP_TY;
    const int t = xcd_local((int)blockIdx.x, (int)gridDim.x);
    const int X0 = (t % gx) * FGP_TX, Y0 = ((t / gx) % gy) * FGP_TY;
    const int Z0 = DIM == 3 ? (t / (gx * gy)) * FGP_ZC : 0;
    const int Z1 = DIM == 3 ? min(nz, Z0 + FGP_ZC) : 1;
    const float w = wstep[0], step = wstep[1];
    const int tx = threadIdx.x % FGP_TX, ty = threadIdx.x / FGP_TX;
    const int X = X0 + tx, Y = Y0 + ty;
    const bool own = X < nx && Y < ny;

    // r of plane z over the tile and its halo into rotation slot z % 3 (zero outside the volume)
    auto build_r = [&](int z) {
        float(*dst)[FGP_HY * FGP_HX] = rL[z % 3];
        for (int e = threadIdx.x; e < FGP_HY * FGP_HX; e += FGP_WG) {
            const int gx = X0 + e % FGP_HX - 1, gy = Y0 + e / FGP_HX - 1;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int64_t o = (int64_t)z * plane + (int64_t)gy * nx + gx;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const float c = pc[a * nvox + o], q = pp[a * nvox + o];
                    dst[a][e] = fmaf(coef, c - q, c);
                }
            } else {
#pragma unroll
                for (int a = 0; a < DIM; ++a) dst[a][e] = 0.0f;
            }
        }
    };

    const int zs = Z0 > 0 ? Z0 - 1 : 0;
    build_r(zs);
    float u_prev = 0.0f;
    for (int z = zs; z < Z1; ++z) {
        if (DIM == 3 && z + 1 < nz) build_r(z + 1);
        __syncthreads();
        // u = b - w D^T r over x, y in [-1, T - 1] (the sums in the order of the
        // separate D^T: +x, -x, +y, -y, +z, -z)
        const float(*rc)[FGP_HY * FGP_HX] = rL[z % 3];
        const float(*rn)[FGP_HY * FGP_HX] = rL[(z + 1) % 3];
        for (int e = threadIdx.x; e < FGP_UY * FGP_UX; e += FGP_WG) {
            const int lx = e % FGP_UX - 1, ly = e / FGP_UX - 1;
            const int gx = X0 + lx, gy = Y0 + ly;
            float uv = 0.0f;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const int h = (ly + 1) * FGP_HX + (lx + 1);
                float d = 0.0f;
                if (gx >= 1) d += rc[0][h];
                if (gx + 1 < nx) d -= rc[0][h + 1];
                if (gy >= 1) d += rc[1][h];
                if (gy + 1 < ny) d -= rc[1][h + FGP_HX];
                if (DIM == 3) {
                    if (z >= 1) d += rc[DIM - 1][h];
                    if (z + 1 < nz) d -= rn[DIM - 1][h];
                }
                uv = b[(int64_t)z * plane + (int64_t)gy * nx + gx] - w * d;
            }
            uL[e] = uv;
        }
        __syncthreads();
        const int hu = (ty + 1) * FGP_UX + (tx + 1);
        const float uc = uL[hu];
        if (own && z >= Z0) {
            float g[3] = {0.0f, 0.0f, 0.0f};
            if (X >= 1) g[0] = uc - uL[hu - 1];
            if (Y >= 1) g[1] = uc - uL[hu - FGP_UX];
            if (DIM == 3 && z >= 1) g[2] = uc - u_prev;
            const int hr = (ty + 1) * FGP_HX + (tx + 1);
            float q[3];
            float n2 = 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                q[a] = fmaf(step, g[a], rc[a][hr]);
                n2 = fmaf(q[a], q[a], n2);
            }
            const float sc = 1.0f / fmaxf(1.0f, sqrtf(n2));
            const int64_t o = (int64_t)z * plane + (int64_t)Y * nx + X;
#pragma unroll
            for (int a = 0; a < DIM; ++a) pn[a * nvox + o] = q[a] * sc;
        }
        u_prev = uc;
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_fgp_final(float* __restrict__ x, const float* __restrict__ p, int nx, int ny,
                                                  int nz, const float* __restrict__ wstep)
{
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t o = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (o >= nvox) return;
    const float w = wstep[0];
    const int X = (int)(o % nx), Y = (int)((o / nx) % ny), Z = (int)(o / ((int64_t)nx * ny));
    x[o] = x[o] - w * div_adj<DIM>(p, nvox, X, Y, Z, nx, ny, nz);
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_geom_stats(const DevGeom& G, double* w, int64_t* nnz, hipStream_t st)
{
    const int64_t waves = (int64_t)G.n_views * G.N;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (G.dim == 3)
        hipLaunchKernelGGL(k_geom_stats<3>, dim3(blocks), dim3(WG), 0, st, G, w, (long long*)nnz);
    else
        hipLaunchKernelGGL(k_geom_stats<2>, dim3(blocks), dim3(WG), 0, st, G, w, (long long*)nnz);
    return hipGetLastError();
}

hipError_t launch_plan(const DevGeom& G, const int32_t* sched, SchedLayout L, int n_iters, uint64_t seed,
                       const uint32_t* q, int64_t im_until, int8_t* draws, PairWork* work, hipStream_t st)
{
    const int64_t per_it = (int64_t)L.maxv * L.B;
    if (n_iters <= 0 || per_it == 0) return hipSuccess;
    for (int it0 = 0; it0 < n_iters; it0 += 65535) {
        const int n = std::min(65535, n_iters - it0);
        hipLaunchKernelGGL(k_plan, dim3(grid1(per_it), n), dim3(WG), 0, st, G, sched, L, it0,
                           (unsigned long long)seed, q, (long long)im_until, draws, work);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Floats of the largest block's LDS copy in the forward projector (2D rows padded).
static int fp_tile_floats(const DevGeom& G)
{
    const int nbx = (G.nx + G.bx - 1) / G.bx + (G.dim == 2 ? 1 : 0);
    return nbx * ((G.ny + G.by - 1) / G.by) * ((G.nz + G.bz - 1) / G.bz);
}

hipError_t launch_fp_pairs(const DevGeom& G, const PairWork* work_it, SchedLayout L, const int32_t* blocks_sel,
                           const float* x, const float* xT, float* z, hipStream_t st)
{
    const int tile = fp_tile_floats(G);
    if (tile <= FP_LDS_MAX_FLOATS) {
        const int chunk = std::max(1, std::min(FP_MAX_CHUNK, G.fp_chunk));
        const unsigned gx = (unsigned)((L.maxv + chunk - 1) / chunk);
        const size_t lds = (size_t)tile * sizeof(float);
        if (G.dim == 3)
            hipLaunchKernelGGL(k_fp_pairs_lds<3>, dim3(gx, L.B), dim3(FP_LDS_WG), lds, st, G, work_it, L, blocks_sel, x, z,
                               chunk);
        else
            hipLaunchKernelGGL(k_fp_pairs_lds<2>, dim3(gx, L.B), dim3(FP_LDS_WG), lds, st, G, work_it, L, blocks_sel, x, z,
                               chunk);
        return hipGetLastError();
    }
    const int64_t waves = (int64_t)L.maxv * L.B * std::max(1, G.fp_wpp);
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (G.dim == 3)
        hipLaunchKernelGGL(k_fp_pairs<3>, dim3(blocks), dim3(WG), 0, st, G, work_it, L, blocks_sel, x, xT, z);
    else
        hipLaunchKernelGGL(k_fp_pairs<2>, dim3(blocks), dim3(WG), 0, st, G, work_it, L, blocks_sel, x, xT, z);
    return hipGetLastError();
}

hipError_t launch_xy_transpose(const float* x, float* xT, int nx, int ny, int nz, hipStream_t st)
{
    if ((int64_t)nx * ny * nz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xy_transpose, dim3((unsigned)((nx + 31) / 32), (unsigned)((ny + 31) / 32), (unsigned)nz),
                       dim3(WG), 0, st, x, xT, nx, ny);
    return hipGetLastError();
}

size_t fp_lds_bytes_for(const DevGeom& G)
{
    const int tile = fp_tile_floats(G);
    return tile <= FP_LDS_MAX_FLOATS ? (size_t)tile * sizeof(float) : 0;
}

size_t resid_lds_bytes_for(const DevGeom& G) { return resid_lds_bytes(G, res_wg(G.dim)); }

static int step_tiles(const DevGeom& G);
static size_t bp_lds_bytes(const DevGeom& G);

void batch_grids(BatchEntry& e)
{
    const DevGeom& G = e.G;
    const SchedLayout& L = e.L;
    if (fp_tile_floats(G) <= FP_LDS_MAX_FLOATS) {
        e.fp_lds = 1;
        e.fp_chunk = std::max(1, std::min(FP_MAX_CHUNK, G.fp_chunk));
        e.gx[0] = (L.maxv + e.fp_chunk - 1) / e.fp_chunk;
    } else {
        e.fp_lds = 0;
        e.fp_chunk = 0;
        e.gx[0] = (int)(((int64_t)L.maxv * L.B * std::max(1, G.fp_wpp) + 3) / 4);
    }
    e.gx[1] = (G.nu * G.nv + res_wg(G.dim) - 1) / res_wg(G.dim);
    e.gx[2] = step_tiles(G);
}

hipError_t launch_batch_iteration(BatchArgs& A, int dim, const int (&wgs)[3], const FpLaunchClass* fp_classes,
                                  int n_fp_classes, const BpLaunchClass* bp_classes, int n_bp_classes,
                                  size_t res_lds, hipStream_t st)
{
    if (A.n == 0) return hipSuccess;
    // forward projection: one launch per LDS size class (contiguous workgroup ranges),
    // so no solve runs with more LDS, and less occupancy, than its own tile needs
    hipError_t e = hipSuccess;
    for (int c = 0; c < n_fp_classes; ++c) {
        const FpLaunchClass& k = fp_classes[c];
        if (k.wgs <= 0) continue;
        A.id0 = k.wg0;
        if (k.lds_bytes > 0) {
            if (dim == 3)
                hipLaunchKernelGGL((k_fp_batch<3, FP_LDS_WG>), dim3(k.wgs), dim3(FP_LDS_WG), k.lds_bytes, st, A);
            else
                hipLaunchKernelGGL((k_fp_batch<2, FP_LDS_WG>), dim3(k.wgs), dim3(FP_LDS_WG), k.lds_bytes, st, A);
        } else if (dim == 3) {
            hipLaunchKernelGGL((k_fp_batch<3, WG>), dim3(k.wgs), dim3(WG), 0, st, A);
        } else {
            hipLaunchKernelGGL((k_fp_batch<2, WG>), dim3(k.wgs), dim3(WG), 0, st, A);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    A.id0 = 0;
    if (dim == 3)
        hipLaunchKernelGGL(k_resid_batch<res_wg(3)>, dim3(wgs[1]), dim3(res_wg(3)), res_lds, st, A);
    else
        hipLaunchKernelGGL(k_resid_batch<res_wg(2)>, dim3(wgs[1]), dim3(res_wg(2)), res_lds, st, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dim == 3) {
        size_t bp_lds = 0;
        for (int i = 0; i < A.n; ++i) bp_lds = std::max(bp_lds, bp_lds_bytes(A.e[i].G));
        hipLaunchKernelGGL(k_bp_batch<3>, dim3(wgs[2]), dim3(bp_wg(3)), bp_lds, st, A);
        return hipGetLastError();
    }
    // 2D back projection: one launch per wave split (contiguous workgroup ranges), each
    // solve with its own tuned workgroup shape
    for (int c = 0; c < n_bp_classes; ++c) {
        const BpLaunchClass& k = bp_classes[c];
        if (k.wgs <= 0) continue;
        A.id0 = k.wg0;
        if (k.split == 2)
            hipLaunchKernelGGL((k_bp_batch<2, 2>), dim3(k.wgs), dim3(bp_wg(2, 2)), 0, st, A);
        else if (k.split == 8)
            hipLaunchKernelGGL((k_bp_batch<2, 8>), dim3(k.wgs), dim3(bp_wg(2, 8)), 0, st, A);
        else
            hipLaunchKernelGGL((k_bp_batch<2>), dim3(k.wgs), dim3(bp_wg(2)), 0, st, A);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    A.id0 = 0;
    return hipSuccess;
}

hipError_t launch_resid(const DevGeom& G, const int32_t* sched_it, SchedLayout L, const float* y, const float* z,
                        float* r_sel, hipStream_t st)
{
    const int per_view = G.nu * G.nv;
    const int tpb = res_wg(G.dim);
    const unsigned gx = (unsigned)((per_view + tpb - 1) / tpb);
    if (G.dim == 3)
        hipLaunchKernelGGL(k_resid<res_wg(3)>, dim3(gx, L.maxv), dim3(tpb), resid_lds_bytes(G, tpb), st, G, sched_it, L,
                           y, z, r_sel);
    else
        hipLaunchKernelGGL(k_resid<res_wg(2)>, dim3(gx, L.maxv), dim3(tpb), resid_lds_bytes(G, tpb), st, G, sched_it, L, y, z,
                       r_sel);
    return hipGetLastError();
}


// Workgroups per block of the back projectors (largest block): 2D pair tiles, 3D
// voxel-column tiles.
static int step_tiles(const DevGeom& G)
{
    if (G.dim == 3) return bp3_tiles(G);
    const int mbx = (G.nx + G.bx - 1) / G.bx, mby = (G.ny + G.by - 1) / G.by;
    return ((mbx + PAIR_TX - 1) / PAIR_TX) * ((mby + PAIR_TY - 1) / PAIR_TY);
}

static size_t bp_lds_bytes(const DevGeom& G) { return G.dim == 3 ? bp3_lds_bytes(G) : 0; }

hipError_t launch_bp_step(const DevGeom& G, const int32_t* sched_it, const PairWork* work_it, SchedLayout L,
                          const float* r_sel, const float* delta, float* ghat, float* gsum, float* x, float* xT,
                          const float* mu, int64_t n_vox, hipStream_t st)
{
    const int tiles = step_tiles(G);
    const dim3 grid(tiles, L.B), blk(bp_wg(G.dim));
    const long long nv = (long long)n_vox;
    const size_t lds = bp_lds_bytes(G);
    if (delta) {
        if (G.dim == 3)
            hipLaunchKernelGGL((k_bp_step<3, true>), grid, blk, lds, st, G, sched_it, work_it, L, delta, ghat, gsum, x,
                               xT, mu, nv);
        else
            hipLaunchKernelGGL((k_bp_step<2, true>), grid, blk, 0, st, G, sched_it, work_it, L, delta, ghat, gsum, x,
                               xT, mu, nv);
    } else if (G.dim == 3) {
        hipLaunchKernelGGL((k_bp_step<3, false>), grid, blk, lds, st, G, sched_it, work_it, L, r_sel, ghat, gsum, x,
                           xT, mu, nv);
    } else if (G.bp_split == 2) {
        hipLaunchKernelGGL((k_bp_step<2, false, 2>), grid, dim3(bp_wg(2, 2)), 0, st, G, sched_it, work_it, L, r_sel,
                           ghat, gsum, x, xT, mu, nv);
    } else if (G.bp_split == 8) {
        hipLaunchKernelGGL((k_bp_step<2, false, 8>), grid, dim3(bp_wg(2, 8)), 0, st, G, sched_it, work_it, L, r_sel,
                           ghat, gsum, x, xT, mu, nv);
    } else {
        hipLaunchKernelGGL((k_bp_step<2, false>), grid, blk, 0, st, G, sched_it, work_it, L, r_sel, ghat, gsum, x,
                           xT, mu, nv);
    }
    return hipGetLastError();
}

hipError_t launch_subdet_delta(const DevGeom& G, const int32_t* sched_it, const PairWork* work_it, SchedLayout L,
                               const float* r_sel, float* rho, float* delta, hipStream_t st)
{
    hipLaunchKernelGGL(k_subdet_delta, dim3(L.maxv, L.B), dim3(WG), 0, st, G, sched_it, work_it, L, r_sel, rho,
                       delta);
    return hipGetLastError();
}

hipError_t launch_fp_full(const DevGeom& G, const int32_t* views, int n_sel, int block, const float* x, float* y,
                          int accumulate, hipStream_t st)
{
    if (n_sel == 0) return hipSuccess;
    const int per_view = G.nu * G.nv;
    const int j0 = block < 0 ? 0 : block, j1 = block < 0 ? G.N : block + 1;
    if (G.dim == 3)
        hipLaunchKernelGGL(k_fp_full<3>, dim3(grid1(per_view), n_sel), dim3(WG), 0, st, G, views, n_sel, j0, j1, x,
                           y, accumulate);
    else
        hipLaunchKernelGGL(k_fp_full<2>, dim3(grid1(per_view), n_sel), dim3(WG), 0, st, G, views, n_sel, j0, j1, x,
                           y, accumulate);
    return hipGetLastError();
}

hipError_t launch_bp_full(const DevGeom& G, const int32_t* views, int n_sel, int block, const float* y, float* x,
                          float scale, int accumulate, hipStream_t st)
{
    const int tiles = step_tiles(G);
    const int j0 = block < 0 ? 0 : block, nj = block < 0 ? G.N : 1;
    if (G.dim == 3)
        hipLaunchKernelGGL(k_bp_full_3d, dim3(tiles, nj), dim3(BP3_WG), bp3_lds_bytes(G), st, G, views, n_sel, j0, y, x,
                           scale, accumulate);
    else
        hipLaunchKernelGGL(k_bp_full_2d, dim3(tiles, nj), dim3(bp_wg(2)), 0, st, G, views, n_sel, j0, y, x, scale,
                           accumulate);
    return hipGetLastError();
}

hipError_t launch_resid_sumsq(const DevGeom& G, const float* y, const float* z, double* partials, int* n_partials,
                              hipStream_t st)
{
    const int per_view = G.nu * G.nv;
    const unsigned gx = grid1(per_view);
    hipLaunchKernelGGL(k_resid_sumsq, dim3(gx, G.n_views), dim3(WG), resid_lds_bytes(G, WG), st, G, y, z, partials);
    *n_partials = (int)(gx * G.n_views);
    return hipGetLastError();
}

hipError_t launch_sumsq(const float* a, int64_t n, double* partials, int* n_partials, hipStream_t st)
{
    int64_t blocks = (n + WG - 1) / WG;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_sumsq, dim3((unsigned)blocks), dim3(WG), 0, st, a, (long long)n, partials);
    *n_partials = (int)blocks;
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partials, int n, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, st, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_sub(const float* b, const float* c, float* a, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub, dim3(grid1(n)), dim3(WG), 0, st, b, c, a, (long long)n);
    return hipGetLastError();
}

hipError_t launch_add(float* a, const float* b, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3(grid1(n)), dim3(WG), 0, st, a, b, (long long)n);
    return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, int64_t n, double* partials, int* n_partials, hipStream_t st)
{
    int64_t blocks = (n + WG - 1) / WG;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_dot, dim3((unsigned)blocks), dim3(WG), 0, st, a, b, (long long)n, partials);
    *n_partials = (int)blocks;
    return hipGetLastError();
}

hipError_t launch_fill(float* a, float v, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(WG), 0, st, a, v, (long long)n);
    return hipGetLastError();
}

void set_bp3_bounds(DevGeom& G, double sod, double sdd, double du, double dv)
{
    G.bp3_kmax = G.bp3_lmax = 0;
    G.bp3_steep = 1;
    if (G.dim != 3) return;
    // a ray's height changes by at most |v| / |(a, b)| <= (nv - 1) dv / (2 sdd) per mm of
    // xy path, and its xy chord through one voxel column is at most the voxel's xy
    // diagonal: below 0.9 vz no chord reaches across a whole voxel, so it meets at
    // most one z plane inside a column (with room for the rounding of the voxel pick)
    {
        const double slope = 0.5 * (G.nv - 1) * dv / sdd;
        const double dxy = std::sqrt((double)G.vx * G.vx + (double)G.vy * G.vy);
        G.bp3_steep = slope * dxy <= 0.9 * (double)G.vz ? 0 : 1;
    }
    // A workgroup tile is at most BP3_TX x BP3_TY x BP3_CZ voxels anywhere in the volume.
    // For two of its points at depths d1, d2 >= dmin and lateral offsets w1, w2,
    // |w1/d1 - w2/d2| <= |w1 - w2| / dmin + |w2| |d1 - d2| / dmin^2, with |w1 - w2| and
    // |d1 - d2| at most the tile's xy diagonal and |w2| at most the volume's xy radius;
    // the same for heights z. The pixel rectangle spans at most that many pixels plus
    // two (integer ends) plus the margins.
    const double vx = G.vx, vy = G.vy, vz = G.vz;
    const double diag = std::sqrt((BP3_TX * vx) * (BP3_TX * vx) + (BP3_TY * vy) * (BP3_TY * vy));
    const double rxy = 0.5 * std::sqrt((G.nx * vx) * (G.nx * vx) + (G.ny * vy) * (G.ny * vy));
    const double zmax = 0.5 * G.nz * vz;
    const double dmin = sod - rxy;
    if (!(dmin > 0.0)) return;
    const double wpx = sdd * (diag / dmin + rxy * diag / (dmin * dmin)) / du;
    const double hpx = sdd * (BP3_CZ * vz / dmin + zmax * diag / (dmin * dmin)) / dv;
    const int km = (int)std::min((double)G.nu, std::floor(wpx) + 3.0);
    const int lm = (int)std::min((double)G.nv, std::floor(hpx) + 3.0);
    DevGeom t = G;
    t.bp3_kmax = km;
    t.bp3_lmax = lm;
    // stay inside the 64 KB a workgroup may address without an opt-in
    if (km > 0 && lm > 0 && bp3_lds_bytes(t) <= 65536) {
        G.bp3_kmax = km;
        G.bp3_lmax = lm;
    }
}

void tv_weight_step(int dim, double mu, double lambda, float* out)
{
    const float w = (float)(mu * lambda);
    out[0] = w;
    out[1] = w > 0.0f ? (float)(1.0 / (4.0 * dim * (double)w)) : 0.0f;
}

hipError_t launch_tv_prox(const DevGeom& G, float* x, const float* wstep, int iters, float* p, float* ra, float* rb,
                          hipStream_t st)
{
    if (iters <= 0) return hipSuccess;
    const int64_t nvox = (int64_t)G.nx * G.ny * G.nz;
    const int dim = G.dim;
    // p_k lives in buf[k % 3]; p_0 = 0 and p_{-1} = p_0
    float* buf[3] = {p, ra, rb};
    hipError_t e = launch_fill(p, 0.0f, dim * nvox, st);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)(((G.nx + FGP_TX - 1) / FGP_TX) * ((G.ny + FGP_TY - 1) / FGP_TY) *
                               (dim == 3 ? (G.nz + FGP_ZC - 1) / FGP_ZC : 1)));
    double tk = 1.0;
    float coef = 0.0f;  // extrapolation weight of the current iterate ((t_{k-1} - 1) / t_k)
    for (int it = 0; it < iters; ++it) {
        const float* pc = buf[it % 3];
        const float* pp = buf[(it + 2) % 3];
        if (it == 0) pp = pc;
        float* pn = buf[(it + 1) % 3];
        if (dim == 3)
            hipLaunchKernelGGL(k_fgp_step<3>, grid, dim3(FGP_WG), 0, st, x, pc, pp, pn, G.nx, G.ny, G.nz, wstep,
                               coef);
        else
            hipLaunchKernelGGL(k_fgp_step<2>, grid, dim3(FGP_WG), 0, st, x, pc, pp, pn, G.nx, G.ny, G.nz, wstep,
                               coef);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const double tn = (1.0 + sqrt(1.0 + 4.0 * tk * tk)) / 2.0;
        coef = (float)((tk - 1.0) / tn);
        tk = tn;
    }
    const float* pf = buf[iters % 3];
    if (dim == 3)
        hipLaunchKernelGGL(k_fgp_final<3>, dim3(grid1(nvox)), dim3(WG), 0, st, x, pf, G.nx, G.ny, G.nz, wstep);
    else
        hipLaunchKernelGGL(k_fgp_final<2>, dim3(grid1(nvox)), dim3(WG), 0, st, x, pf, G.nx, G.ny, G.nz, wstep);
    return hipGetLastError();
}

}  // namespace bsgd
