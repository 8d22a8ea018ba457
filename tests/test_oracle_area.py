"""Pins of the oracle's projected-area importance weights (Sec. II-A, Algorithm 2):
brute-force shadows (rays through a fine grid of detector points tested against the
block's box), the closed-form parallel-beam shadow length, fractions that add up to
one when the shadow lies on the detector, and weight one for a shadow on a single
sub-detector."""
import math

import numpy as np

from bsgd_inputs.configs import GeometrySpec
from oracle.area import area_weights, block_boxes, corner_pixels, subdetector_rect
from oracle.bsgd import quantise

CONE = GeometrySpec(kind="cone3d", nx=20, ny=18, nz=14, vx=1.0, vy=1.0, vz=0.947, n_views=7,
                    angle_span=2 * math.pi, nu=40, nv=30, du=1.3, dv=1.2373, sod=40.0, sdd=90.0,
                    bx=2, by=3, bz=2, n_row_blocks=1, partition_seed=3, su=2, sv=2, im_mode="area")
FAN = GeometrySpec(kind="fan2d", nx=41, ny=35, nz=1, vx=0.8, vy=0.8, vz=0.8, n_views=9,
                   angle_span=2 * math.pi, nu=64, nv=1, du=1.1, dv=1.0, sod=60.0, sdd=130.0,
                   bx=3, by=3, bz=1, n_row_blocks=1, partition_seed=4, su=3, sv=1, im_mode="area")
PAR = GeometrySpec(kind="parallel2d", nx=30, ny=22, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=11,
                   angle_span=math.pi, nu=80, nv=1, du=0.9, dv=1.0, bx=2, by=2, bz=1,
                   n_row_blocks=1, partition_seed=5, su=4, sv=1, im_mode="area")


def _ray_hits_box(src, pts, lo, hi):
    """Slab test of the segments src -> pts[i] (extended to a line) against a box."""
    d = pts - src
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (np.asarray(lo) - src) * inv
        t1 = (np.asarray(hi) - src) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    return tmax > np.maximum(tmin, 0.0)


def _brute_area(g, view, box, rect, step):
    th = g.angles()[view]
    c, s = math.cos(th), math.sin(th)
    x0, x1, y0, y1 = rect
    ks = np.arange(x0 + step / 2, x1, step)
    ls = np.arange(y0 + step / 2, y1, step) if g.is_3d else np.array([0.0])
    K, L = np.meshgrid(ks, ls, indexing="ij")
    u = (K.ravel() - (g.nu - 1) / 2.0) * g.du
    src = np.array([g.sod * c, g.sod * s] + ([0.0] if g.is_3d else []))
    det = np.stack([-(g.sdd - g.sod) * c - u * s, -(g.sdd - g.sod) * s + u * c], axis=1)
    if g.is_3d:
        v = (L.ravel() - (g.nv - 1) / 2.0) * g.dv
        det = np.concatenate([det, v[:, None]], axis=1)
    hits = _ray_hits_box(src, det, box[0], box[1])
    return hits.sum() * step * (step if g.is_3d else 1.0)


def test_cone_areas_match_brute_force_shadows():
    w = area_weights(CONE)
    boxes = block_boxes(CONE)
    checked = 0
    for v in (0, 3):
        for j in (0, 5, 11):
            for sd in range(4):
                ref = _brute_area(CONE, v, boxes[j], subdetector_rect(CONE, sd), 0.04)
                assert abs(w[v, sd, j] - ref) <= 0.02 * max(ref, 1.0), (v, j, sd, w[v, sd, j], ref)
                checked += ref > 0
    assert checked >= 6


def test_fan_lengths_match_brute_force_shadows():
    w = area_weights(FAN)
    boxes = block_boxes(FAN)
    for v in (0, 4, 7):
        for j in range(9):
            for sd in range(3):
                ref = _brute_area(FAN, v, boxes[j], subdetector_rect(FAN, sd), 0.002)
                assert abs(w[v, sd, j] - ref) <= 0.005, (v, j, sd, w[v, sd, j], ref)


def test_parallel_shadow_length_closed_form():
    # a W x H block seen at angle t spans W |sin t| + H |cos t| along the detector
    w = area_weights(PAR)
    boxes = block_boxes(PAR)
    for v, t in enumerate(PAR.angles()):
        for j, (lo, hi) in enumerate(boxes):
            W, H = hi[0] - lo[0], hi[1] - lo[1]
            length = (W * abs(math.sin(t)) + H * abs(math.cos(t))) / PAR.du
            P = corner_pixels(PAR, v, (lo, hi))
            if P[:, 0].min() >= -0.5 and P[:, 0].max() <= PAR.nu - 0.5:
                assert abs(w[v, :, j].sum() - length) <= 1e-9 * length


def test_fractions_sum_to_one_and_single_subdetector_weight():
    from scipy.spatial import ConvexHull
    w = area_weights(CONE)
    boxes = block_boxes(CONE)
    full = 0
    for v in range(CONE.n_views):
        for j, box in enumerate(boxes):
            P = corner_pixels(CONE, v, box)
            inside = (P[:, 0].min() >= -0.5 and P[:, 0].max() <= CONE.nu - 0.5 and
                      P[:, 1].min() >= -0.5 and P[:, 1].max() <= CONE.nv - 0.5)
            if inside:
                full += 1
                assert abs(w[v, :, j].sum() - ConvexHull(P).volume) <= 1e-9 * ConvexHull(P).volume
    assert full > 20
    # a small block near the axis whose shadow lies inside one quadrant sub-detector
    g = GeometrySpec(kind="cone3d", nx=16, ny=16, nz=16, vx=1.0, vy=1.0, vz=1.0, n_views=4,
                     angle_span=2 * math.pi, nu=40, nv=40, du=1.5, dv=1.5, sod=40.0, sdd=90.0,
                     bx=4, by=4, bz=4, n_row_blocks=1, partition_seed=3, su=2, sv=2, im_mode="area")
    q = quantise(area_weights(g))
    hit = 0
    for v in range(g.n_views):
        for j in range(g.n_blocks):
            nz = np.flatnonzero(q[v, :, j])
            if len(nz) == 1:
                assert q[v, nz[0], j] == 1 << 20
                hit += 1
    assert hit > 0
