"""Pins of the oracle's system matrix (Siddon lengths) against independent facts."""
import json
import math
import os

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec, ray_count, voxel_count
from oracle import geometry as geo
from oracle.siddon import siddon_ray, brute_force_row, voxel_boxes, slab_length
from oracle.system import matrix_python, matrix
from oracle.cfast import Projector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def _random_rays(rng, grid, n):
    ext = np.array([ni * vi for ni, vi in zip(grid.n, grid.v)])
    lo = np.array(grid.lo)
    p0 = lo + rng.uniform(-0.5, 1.5, size=(n, grid.dim)) * ext
    p1 = lo + rng.uniform(-0.5, 1.5, size=(n, grid.dim)) * ext
    return p0, p1


@pytest.mark.parametrize("dims", [((7, 5), (0.7, 1.3)), ((5, 4, 3), (0.9, 1.1, 0.6))])
def test_siddon_matches_brute_force(dims):
    n, v = dims
    grid = geo.Grid(n=n, lo=tuple(-0.5 * a * b for a, b in zip(n, v)), v=v)
    boxes = voxel_boxes(grid)
    rng = np.random.Generator(np.random.PCG64(7))
    p0, p1 = _random_rays(rng, grid, 300)
    for i in range(p0.shape[0]):
        dense = np.zeros(int(np.prod(n)))
        idx, ln = siddon_ray(p0[i], p1[i], grid)
        np.add.at(dense, idx, ln)
        ref = brute_force_row(p0[i], p1[i], grid, boxes)
        assert np.allclose(dense, ref, rtol=0, atol=1e-12), i


def test_row_sum_is_chord_through_grid_box():
    g = GeometrySpec(kind="fan2d", nx=20, ny=14, nz=1, vx=1.5, vy=1.5, vz=1.5, n_views=7,
                     angle_span=2 * math.pi, nu=40, nv=1, du=1.0, dv=1.0, sod=40.0, sdd=80.0)
    A = matrix_python(g)
    p0, p1 = geo.ray_endpoints(g)
    grid = geo.grid_of(g)
    lo = np.array(grid.lo)[None]
    hi = lo + np.array([a * b for a, b in zip(grid.n, grid.v)])[None]
    chords = np.array([slab_length(p0[i], p1[i], lo, hi)[0] for i in range(p0.shape[0])])
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), chords, atol=1e-11)
    assert chords.max() > 0


def test_parallel_opposite_views_reverse_bins():
    g = GeometrySpec(kind="parallel2d", nx=12, ny=12, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=8,
                     angle_span=2 * math.pi, nu=18, nv=1, du=0.9, dv=1.0)
    A = matrix_python(g).toarray().reshape(g.n_views, g.nu, -1)
    half = g.n_views // 2
    for m in range(half):
        assert np.allclose(A[m], A[m + half][::-1], atol=1e-12)


@pytest.mark.parametrize("g", [
    GeometrySpec(kind="parallel2d", nx=9, ny=11, nz=1, vx=1.0, vy=0.8, vz=1.0, n_views=6,
                 angle_span=math.pi, nu=15, nv=1, du=0.9, dv=1.0),
    GeometrySpec(kind="fan2d", nx=10, ny=10, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=9,
                 angle_span=2 * math.pi, nu=17, nv=1, du=1.1, dv=1.0, sod=30.0, sdd=60.0),
    GeometrySpec(kind="cone3d", nx=6, ny=5, nz=4, vx=1.0, vy=1.2, vz=0.9, n_views=5,
                 angle_span=2 * math.pi, nu=9, nv=7, du=1.3, dv=1.1, sod=25.0, sdd=50.0),
])
def test_c_restatement_matches_python(g):
    A_py = matrix_python(g)
    A_c = matrix(g)
    assert A_py.shape == A_c.shape
    assert abs(A_py - A_c).max() < 1e-12
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.uniform(size=A_py.shape[1])
    r = rng.normal(size=A_py.shape[0])
    P = Projector(g)
    assert np.allclose(P.fp(x), A_py @ x, rtol=0, atol=1e-11)
    assert np.allclose(P.bp(r, threads=3), A_py.T @ r, rtol=0, atol=1e-11)
    assert P.last_nnz == A_py.nnz


def test_paper_matrix_sizes():
    gold = json.load(open(GOLDEN))["matrix_sizes"]
    e1 = gold[0]
    g = GeometrySpec(kind="fan2d", nx=e1["nx"], ny=e1["ny"], nz=1, vx=1.0, vy=1.0, vz=1.0,
                     n_views=e1["n_views"], angle_span=2 * math.pi, nu=e1["nu"], nv=1, du=1.0,
                     dv=1.0, sod=50.0, sdd=100.0)
    A = matrix_python(g)
    assert A.shape == (e1["rows"], e1["cols"])
    for case in gold[1:]:
        g = GeometrySpec(kind="cone3d", nx=case["nx"], ny=case["nx"], nz=case["nx"], vx=1, vy=1, vz=1,
                         n_views=case["n_views"], angle_span=2 * math.pi, nu=case["nu"],
                         nv=case["nv"], du=1, dv=1, sod=1000.0, sdd=1536.0)
        # the exact counts, rounded to the precision the paper prints, equal the printed values
        for count, printed in ((ray_count(g), case["rows_approx"]), (voxel_count(g), case["cols_approx"])):
            mant = printed.split("e")[0]
            digits = len(mant.split(".")[1]) if "." in mant else 0
            assert f"{count:.{digits}e}".replace("e+0", "e") == printed


def _ellipse_line_integral(p0, p1, cx, cy, a, b, ang, val):
    """Closed-form chord of a line with a filled ellipse (roots of the quadratic), times density."""
    d = p1 - p0
    L = np.linalg.norm(d)
    d = d / L
    c, s = math.cos(ang), math.sin(ang)
    e1 = np.array([c, s])
    e2 = np.array([-s, c])
    q = p0 - np.array([cx, cy])
    A2 = (d @ e1) ** 2 / a ** 2 + (d @ e2) ** 2 / b ** 2
    B2 = 2 * ((q @ e1) * (d @ e1) / a ** 2 + (q @ e2) * (d @ e2) / b ** 2)
    C2 = (q @ e1) ** 2 / a ** 2 + (q @ e2) ** 2 / b ** 2 - 1
    disc = B2 * B2 - 4 * A2 * C2
    return val * math.sqrt(disc) / A2 if disc > 0 else 0.0


def test_fp_of_pixelised_ellipses_converges_to_analytic_radon():
    shapes = [(10.0, -6.0, 20.0, 12.0, 0.4, 1.0), (-15.0, 8.0, 9.0, 14.0, 1.9, 0.5)]
    errs = []
    for n in (32, 64, 128):
        v = 64.0 / n
        g = GeometrySpec(kind="fan2d", nx=n, ny=n, nz=1, vx=v, vy=v, vz=v, n_views=24,
                         angle_span=2 * math.pi, nu=64, nv=1, du=2.0, dv=1.0, sod=100.0, sdd=200.0)
        c = (np.arange(n) - (n - 1) / 2) * v
        X, Y = np.meshgrid(c, c)
        img = np.zeros((n, n))
        for cx, cy, a, b, ang, val in shapes:
            cs, sn = math.cos(ang), math.sin(ang)
            u = (cs * (X - cx) + sn * (Y - cy)) / a
            w = (-sn * (X - cx) + cs * (Y - cy)) / b
            img[u * u + w * w <= 1] += val
        P = Projector(g)
        y = P.fp(img.ravel())
        ya = np.array([sum(_ellipse_line_integral(P.p0[i], P.p1[i], *sh) for sh in shapes)
                       for i in range(P.n_rays)])
        errs.append(np.linalg.norm(y - ya) / np.linalg.norm(ya))
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[2] < 0.6 * errs[0]
    assert errs[2] < 0.02


def _ellipsoid_line_integral(p0, p1, centre, semi, R, val):
    """Closed-form chord of a line with a filled ellipsoid {c + R u : sum (u_i / s_i)^2 <= 1}
    (roots of the quadratic along the line), times density."""
    d = p1 - p0
    d = d / np.linalg.norm(d)
    q = R.T @ (p0 - centre)
    e = R.T @ d
    s2 = np.asarray(semi) ** 2
    A2 = np.sum(e * e / s2)
    B2 = 2 * np.sum(q * e / s2)
    C2 = np.sum(q * q / s2) - 1
    disc = B2 * B2 - 4 * A2 * C2
    return val * math.sqrt(disc) / A2 if disc > 0 else 0.0


def _rotation(a, b, c):
    """Rotation R_z(a) R_y(b) R_x(c)."""
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rx = np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]])
    return Rz @ Ry @ Rx


def test_fp_of_voxelised_ellipsoids_converges_to_analytic_line_integrals():
    # the 3D counterpart of the ellipse pin: cone-beam rays through point-sampled
    # ellipsoids approach the exact line integrals as the voxels shrink
    shapes = [(np.array([6.0, -4.0, 3.0]), (14.0, 9.0, 7.0), _rotation(0.4, 0.3, -0.2), 1.0),
              (np.array([-9.0, 7.0, -5.0]), (6.0, 10.0, 8.0), _rotation(1.9, -0.5, 0.7), 0.5)]
    errs = []
    for n in (16, 32, 64):
        v = 48.0 / n
        g = GeometrySpec(kind="cone3d", nx=n, ny=n, nz=n, vx=v, vy=v, vz=v, n_views=6,
                         angle_span=2 * math.pi, nu=24, nv=24, du=4.0, dv=4.0, sod=100.0, sdd=200.0)
        c = (np.arange(n) - (n - 1) / 2) * v
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        pts = np.stack([X, Y, Z], axis=-1)
        img = np.zeros((n, n, n))
        for centre, semi, R, val in shapes:
            u = (pts - centre) @ R  # coordinates in the ellipsoid's axes
            img[np.sum((u / np.asarray(semi)) ** 2, axis=-1) <= 1] += val
        P = Projector(g)
        y = P.fp(img.ravel())
        ya = np.array([sum(_ellipsoid_line_integral(P.p0[i], P.p1[i], *sh) for sh in shapes)
                       for i in range(P.n_rays)])
        errs.append(np.linalg.norm(y - ya) / np.linalg.norm(ya))
    # first order in the voxel size (point-sampled boundaries): about halved per halving;
    # a swapped axis or a wrong rotation leaves an error that does not shrink
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]
    assert errs[2] < 0.07
