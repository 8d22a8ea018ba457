"""Importance weights of BSGD-IM from projected areas.

TEST INFRASTRUCTURE (oracle), FP64.

Sec. II-A (Algorithm 2) estimates how dense the sub-matrix of a column block J_j and
a sub-detector is by the share of the block's projection that falls on that
sub-detector. Here, for view v, block j and sub-detector s:

  w[v][s][j] = area of (shadow of block j in view v) intersected with the rectangle
               of sub-detector s,

in detector pixel units (pixel k covers [k - 1/2, k + 1/2], so sub-detector pixels
[k0, k1) cover [k0 - 1/2, k1 - 1/2]). The shadow of a box is the set of detector
points whose ray meets the box; for a central projection (fan, cone) and for a
parallel one it is the convex hull of the projections of the box's corners. In 2D
the shadow is an interval and its "area" is its length.

The intersection of two convex polygons is the convex hull of the vertices of each
that lie inside the other and of the crossings of their edges; its area is that
hull's (scipy's Qhull gives the hull).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import ConvexHull

from bsgd_inputs.configs import GeometrySpec
from . import geometry as geo


def corner_pixels(g: GeometrySpec, view: int, box) -> np.ndarray:
    """Continuous detector coordinates (k, l) of the corners of box = (lo, hi) (mm)."""
    lo, hi = box
    th = g.angles()[view]
    c, s = np.cos(th), np.sin(th)
    ku, lv = (g.nu - 1) / 2.0, (g.nv - 1) / 2.0
    out = []
    dims = 3 if g.is_3d else 2
    for q in range(1 << dims):
        p = [hi[a] if (q >> a) & 1 else lo[a] for a in range(dims)]
        w = -p[0] * s + p[1] * c  # offset along the detector u axis
        if g.kind == "parallel2d":
            out.append((w / g.du + ku, 0.0))
            continue
        depth = g.sod - (p[0] * c + p[1] * s)  # distance from the source along the central ray
        k = g.sdd * w / depth / g.du + ku
        l = g.sdd * p[2] / depth / g.dv + lv if g.is_3d else 0.0
        out.append((k, l))
    return np.array(out)


def _inside(eqs, pts, tol=1e-12):
    return np.all(pts @ eqs[:, :2].T + eqs[:, 2] <= tol, axis=1)


def _segment_crossings(P, Q):
    """Crossing points of the edges of closed polygons P and Q (vertex arrays)."""
    out = []
    for i in range(len(P)):
        a, b = P[i], P[(i + 1) % len(P)]
        for j in range(len(Q)):
            c, d = Q[j], Q[(j + 1) % len(Q)]
            r, t = b - a, d - c
            den = r[0] * t[1] - r[1] * t[0]
            if den == 0.0:
                continue
            u = ((c[0] - a[0]) * t[1] - (c[1] - a[1]) * t[0]) / den
            v = ((c[0] - a[0]) * r[1] - (c[1] - a[1]) * r[0]) / den
            if 0.0 <= u <= 1.0 and 0.0 <= v <= 1.0:
                out.append(a + u * r)
    return out


def convex_overlap_area(P: np.ndarray, rect) -> float:
    """Area of conv(P) intersected with the rectangle rect = (x0, x1, y0, y1)."""
    x0, x1, y0, y1 = rect
    R = np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]])
    hp = ConvexHull(P)
    hr = ConvexHull(R)
    Pv = P[hp.vertices]
    pts = [p for p in Pv[_inside(hr.equations, Pv)]]
    pts += [r for r in R[_inside(hp.equations, R)]]
    pts += _segment_crossings(Pv, R)
    if len(pts) < 3:
        return 0.0
    pts = np.array(pts)
    if np.linalg.matrix_rank(pts - pts[0], tol=1e-12) < 2:
        return 0.0
    return float(ConvexHull(pts).volume)


def block_boxes(g: GeometrySpec):
    """(lo, hi) corners (mm) of every column block, in block order."""
    grid = geo.grid_of(g)
    bounds = [geo.tile_bounds(g.nx, g.bx), geo.tile_bounds(g.ny, g.by)]
    if g.is_3d:
        bounds.append(geo.tile_bounds(g.nz, g.bz))
    boxes = []
    zs = bounds[2] if g.is_3d else [(0, 1)]
    for (z0, z1) in zs:
        for (y0, y1) in bounds[1]:
            for (x0, x1) in bounds[0]:
                idx0 = (x0, y0, z0)[:grid.dim]
                idx1 = (x1, y1, z1)[:grid.dim]
                lo = [grid.lo[a] + idx0[a] * grid.v[a] for a in range(grid.dim)]
                hi = [grid.lo[a] + idx1[a] * grid.v[a] for a in range(grid.dim)]
                boxes.append((lo, hi))
    return boxes


def subdetector_rect(g: GeometrySpec, sd: int):
    a, b = sd % g.su, sd // g.su
    k0, k1 = (a * g.nu) // g.su, ((a + 1) * g.nu) // g.su
    l0, l1 = (b * g.nv) // g.sv, ((b + 1) * g.nv) // g.sv
    return (k0 - 0.5, k1 - 0.5, l0 - 0.5, l1 - 0.5)


def area_weights(g: GeometrySpec) -> np.ndarray:
    """w[v][s][j]: projected area of block j on sub-detector s of view v (pixels^2; 2D: pixels)."""
    S = g.su * g.sv
    boxes = block_boxes(g)
    w = np.zeros((g.n_views, S, len(boxes)))
    for v in range(g.n_views):
        for j, box in enumerate(boxes):
            P = corner_pixels(g, v, box)
            for sd in range(S):
                x0, x1, y0, y1 = subdetector_rect(g, sd)
                if g.is_3d:
                    w[v, sd, j] = convex_overlap_area(P, (x0, x1, y0, y1))
                else:
                    a, b = P[:, 0].min(), P[:, 0].max()
                    w[v, sd, j] = max(0.0, min(b, x1) - max(a, x0))
    return w
