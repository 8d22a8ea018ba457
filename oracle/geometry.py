"""Scan geometry, ray endpoints and the block partitions of the system matrix.

TEST INFRASTRUCTURE (oracle), FP64.

* Rays (Sec. I: y = A x + e; Fig. 3 scanning geometry): each detector pixel
  defines one row of A. Fan/cone rays are the segment from the source to the
  detector-pixel centre; parallel rays are lines, represented by a segment long
  enough to cross the whole grid.
* Row blocks I_i (Sec. II, Eq. (e1)): groups of whole views. The paper's 3D
  experiment partitions the projections at random into groups (Sec. III-E); here
  a seeded Fisher-Yates permutation of the view indices is cut into M consecutive
  chunks (the first n mod M chunks one view longer), views ascending in a group.
* Column blocks J_j (Eq. (e1), Fig. 2): a regular bx x by x bz tiling of the grid.
* Sub-detectors (Fig. 2, Algorithm 2): su x sv tiles of each view's detector.

The conventions (axes, centres, orderings) are the ones stated in
``bsgd_inputs.configs``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from bsgd_inputs.configs import GeometrySpec
from . import rng


@dataclass
class Grid:
    n: tuple      # voxels per axis (x, y[, z])
    lo: tuple     # lower corner per axis
    v: tuple      # voxel size per axis

    @property
    def dim(self):
        return len(self.n)


def grid_of(g: GeometrySpec) -> Grid:
    if g.is_3d:
        n = (g.nx, g.ny, g.nz)
        v = (g.vx, g.vy, g.vz)
    else:
        n = (g.nx, g.ny)
        v = (g.vx, g.vy)
    lo = tuple(-0.5 * ni * vi for ni, vi in zip(n, v))
    return Grid(n=n, lo=lo, v=v)


def detector_u(g: GeometrySpec) -> np.ndarray:
    return (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.du


def detector_v(g: GeometrySpec) -> np.ndarray:
    return (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.dv


def ray_endpoints(g: GeometrySpec, rays=None):
    """Return (p0, p1), each [n, dim] float64, for all rays ([view][v][u] order) or a subset."""
    per_view = g.nu * g.nv
    idx = np.arange(g.n_views * per_view) if rays is None else np.asarray(rays, dtype=np.int64)
    m = idx // per_view
    l = (idx // g.nu) % g.nv
    k = idx % g.nu
    th = g.angles()[m]
    c, s = np.cos(th), np.sin(th)
    u = (k - (g.nu - 1) / 2.0) * g.du
    if g.kind == "parallel2d":
        grid = grid_of(g)
        reach = math.hypot(*[ni * vi for ni, vi in zip(grid.n, grid.v)]) + 10.0
        q = np.stack([-u * s, u * c], axis=1)
        e = np.stack([c, s], axis=1)
        return q - reach * e, q + reach * e
    if g.kind == "fan2d":
        src = np.stack([g.sod * c, g.sod * s], axis=1)
        det = np.stack([-(g.sdd - g.sod) * c - u * s, -(g.sdd - g.sod) * s + u * c], axis=1)
        return src, det
    v = (l - (g.nv - 1) / 2.0) * g.dv
    src = np.stack([g.sod * c, g.sod * s, np.zeros_like(c)], axis=1)
    det = np.stack([-(g.sdd - g.sod) * c - u * s, -(g.sdd - g.sod) * s + u * c, v], axis=1)
    return src, det


def tile_bounds(n: int, b: int) -> List[tuple]:
    return [((t * n) // b, ((t + 1) * n) // b) for t in range(b)]


def column_blocks(g: GeometrySpec) -> List[np.ndarray]:
    """Voxel indices ([z][y][x] flattening) of each column block J_j, j = (tz by + ty) bx + tx."""
    bxs, bys, bzs = tile_bounds(g.nx, g.bx), tile_bounds(g.ny, g.by), tile_bounds(g.nz, g.bz)
    out = []
    for (z0, z1) in bzs:
        for (y0, y1) in bys:
            for (x0, x1) in bxs:
                zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1),
                                         indexing="ij")
                out.append(((zz * g.ny + yy) * g.nx + xx).reshape(-1))
    return out


def view_groups(g: GeometrySpec) -> List[List[int]]:
    """The M row blocks as lists of view indices (ascending within a group)."""
    perm = rng.permutation(g.partition_seed, rng.STREAM_PARTITION, g.n_views)
    M = g.n_row_blocks
    base, extra = divmod(g.n_views, M)
    groups, pos = [], 0
    for i in range(M):
        size = base + (1 if i < extra else 0)
        groups.append(sorted(perm[pos:pos + size]))
        pos += size
    return groups


def rays_of_view(g: GeometrySpec, view: int) -> np.ndarray:
    per = g.nu * g.nv
    return np.arange(view * per, (view + 1) * per)


def subdetector_rays(g: GeometrySpec, view: int, s: int) -> np.ndarray:
    """Ray indices of sub-detector s = b * su + a (a along u, b along v) of a view."""
    a, b = s % g.su, s // g.su
    k0, k1 = (a * g.nu) // g.su, ((a + 1) * g.nu) // g.su
    l0, l1 = (b * g.nv) // g.sv, ((b + 1) * g.nv) // g.sv
    L, K = np.meshgrid(np.arange(l0, l1), np.arange(k0, k1), indexing="ij")
    return (view * g.nv * g.nu + L * g.nu + K).reshape(-1)


def rays_of_group(g: GeometrySpec, views) -> np.ndarray:
    return np.concatenate([rays_of_view(g, v) for v in views])
