"""Exact ray/voxel intersection lengths: the entries a_ij of the system matrix.

TEST INFRASTRUCTURE (oracle), FP64.

The paper builds A with Siddon's method (Sec. I, after Eq. (yax), citing the
improved Siddon algorithm of Jacobs et al. 1998): a_ij is the length of ray i
inside voxel j. ``siddon_ray`` is the classic parametric formulation: write the
ray as p0 + alpha (p1 - p0), alpha in [0, 1]; collect the alpha values where the
ray meets every grid plane inside the grid; sort and merge them; each pair of
consecutive values bounds one segment, whose voxel is found from its midpoint and
whose length is the alpha difference times |p1 - p0|.

Ties (reading of an unstated detail): voxels are half-open [lo + i v, lo + (i+1) v);
zero-length segments (a ray through a corner) are dropped; an axis along which the
ray does not move contributes no planes and the ray must lie inside that slab.

``slab_length`` is an independent second method (clip the ray against one voxel
box), used as a brute-force check on small grids.

Pinned by: brute-force agreement, analytic chord length of the whole grid box,
parallel-beam opposite-view symmetry, analytic line integrals of ellipses.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Grid


def siddon_ray(p0, p1, grid: Grid):
    """(voxel indices, lengths) of the ray p0 -> p1 through the grid, in order along the ray."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    d = p1 - p0
    length = math.sqrt(float(np.dot(d, d)))
    dim = grid.dim
    amin, amax = 0.0, 1.0
    for ax in range(dim):
        lo = grid.lo[ax]
        hi = lo + grid.n[ax] * grid.v[ax]
        if d[ax] != 0.0:
            a0 = (lo - p0[ax]) / d[ax]
            a1 = (hi - p0[ax]) / d[ax]
            amin = max(amin, min(a0, a1))
            amax = min(amax, max(a0, a1))
        elif not (lo <= p0[ax] < hi):
            return np.zeros(0, dtype=np.int64), np.zeros(0)
    if not amin < amax:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    alphas = [np.array([amin, amax])]
    for ax in range(dim):
        if d[ax] != 0.0:
            planes = grid.lo[ax] + np.arange(grid.n[ax] + 1) * grid.v[ax]
            a = (planes - p0[ax]) / d[ax]
            alphas.append(a[(a > amin) & (a < amax)])
    a = np.unique(np.concatenate(alphas))
    da = np.diff(a)
    mid = 0.5 * (a[:-1] + a[1:])
    keep = da > 0
    mid, da = mid[keep], da[keep]
    flat = np.zeros(mid.shape, dtype=np.int64)
    stride = 1
    for ax in range(dim):
        coord = p0[ax] + mid * d[ax]
        i = np.floor((coord - grid.lo[ax]) / grid.v[ax]).astype(np.int64)
        i = np.clip(i, 0, grid.n[ax] - 1)
        flat += i * stride
        stride *= grid.n[ax]
    return flat, da * length


def slab_length(p0, p1, box_lo, box_hi):
    """Length of the segment p0 -> p1 inside the closed box [box_lo, box_hi] (slab clipping).

    Vectorised over boxes: box_lo / box_hi are [n_boxes, dim].
    """
    p0 = np.asarray(p0, dtype=np.float64)
    d = np.asarray(p1, dtype=np.float64) - p0
    length = math.sqrt(float(np.dot(d, d)))
    box_lo = np.atleast_2d(box_lo)
    box_hi = np.atleast_2d(box_hi)
    t0 = np.zeros(box_lo.shape[0])
    t1 = np.ones(box_lo.shape[0])
    for ax in range(box_lo.shape[1]):
        if d[ax] != 0.0:
            a = (box_lo[:, ax] - p0[ax]) / d[ax]
            b = (box_hi[:, ax] - p0[ax]) / d[ax]
            t0 = np.maximum(t0, np.minimum(a, b))
            t1 = np.minimum(t1, np.maximum(a, b))
        else:
            inside = (box_lo[:, ax] <= p0[ax]) & (p0[ax] < box_hi[:, ax])
            t1 = np.where(inside, t1, -np.inf)
    return np.maximum(t1 - t0, 0.0) * length


def voxel_boxes(grid: Grid):
    """[c, dim] lower and upper corners of every voxel, flattened x fastest."""
    axes = [grid.lo[ax] + np.arange(grid.n[ax]) * grid.v[ax] for ax in range(grid.dim)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")  # slowest axis first
    lo = np.stack([m.reshape(-1) for m in reversed(mesh)], axis=1)
    hi = lo + np.asarray(grid.v)[None, :]
    return lo, hi


def brute_force_row(p0, p1, grid: Grid, boxes=None):
    """Dense row of A by clipping the ray against every voxel separately."""
    lo, hi = boxes if boxes is not None else voxel_boxes(grid)
    return slab_length(p0, p1, lo, hi)
