"""Shared test utilities: small parity geometries, oracle caches, error metrics."""
from __future__ import annotations

import functools
import math
import sys

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec


def log(msg: str):
    """Name the case on stdout before a GPU step (flushed, so a crash still shows it)."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Small geometries: several column blocks with uneven tiles, view counts not divisible
# by M, no ray lying exactly on a grid plane.
PARALLEL_SMALL = GeometrySpec(kind="parallel2d", nx=37, ny=29, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=31,
                              angle_span=math.pi, nu=48, nv=1, du=0.9, dv=1.0, bx=3, by=2, bz=1,
                              n_row_blocks=4, partition_seed=21)
FAN_SMALL = GeometrySpec(kind="fan2d", nx=41, ny=35, nz=1, vx=0.8, vy=0.8, vz=0.8, n_views=40,
                         angle_span=2 * math.pi, nu=64, nv=1, du=1.1, dv=1.0, sod=60.0, sdd=130.0,
                         bx=3, by=3, bz=1, n_row_blocks=5, partition_seed=22, su=3, sv=1)
CONE_SMALL = GeometrySpec(kind="cone3d", nx=20, ny=18, nz=14, vx=1.0, vy=1.0, vz=0.947, n_views=24,
                          angle_span=2 * math.pi, nu=28, nv=22, du=1.3, dv=1.2373, sod=40.0, sdd=90.0,
                          bx=2, by=3, bz=2, n_row_blocks=4, partition_seed=23, su=2, sv=2)
# blocks larger than the forward projector's 64 KB LDS stage (global-memory path)
FAN_WIDE = GeometrySpec(kind="fan2d", nx=262, ny=260, nz=1, vx=0.3, vy=0.3, vz=0.3, n_views=30,
                        angle_span=2 * math.pi, nu=180, nv=1, du=1.1, dv=1.0, sod=90.0, sdd=200.0,
                        bx=2, by=2, bz=1, n_row_blocks=3, partition_seed=24)
CONE_WIDE = GeometrySpec(kind="cone3d", nx=66, ny=64, nz=26, vx=0.5, vy=0.5, vz=0.47, n_views=16,
                         angle_span=2 * math.pi, nu=44, nv=30, du=1.3, dv=1.2373, sod=60.0, sdd=130.0,
                         bx=2, by=2, bz=1, n_row_blocks=4, partition_seed=25)
SMALL = {"parallel": PARALLEL_SMALL, "fan": FAN_SMALL, "cone": CONE_SMALL, "fan_wide": FAN_WIDE,
         "cone_wide": CONE_WIDE}


@functools.lru_cache(maxsize=16)
def oracle_matrix(g: GeometrySpec):
    from oracle.system import matrix
    return matrix(g)


@functools.lru_cache(maxsize=16)
def oracle_problem(g: GeometrySpec):
    from oracle.bsgd import Problem
    return Problem.build(g, oracle_matrix(g))


@functools.lru_cache(maxsize=4)
def oracle_study(name: str):
    """A 2D study setup of the paper on the oracle: (problem with one block, y, x_true,
    x_lsq, ||A||_2^2), y = A x_true + white noise at the setup's data SNR; x_lsq (dense
    least squares) only for the 16x16 setup, else None."""
    from bsgd_inputs.configs import STUDY_2D, study_geometry
    from bsgd_inputs.phantoms import add_gaussian_noise_snr, ellipse_phantom_2d
    from oracle.bsgd import lipschitz
    d = STUDY_2D[name]
    p = oracle_problem(study_geometry(name, 1, 1, 1))
    x_true = ellipse_phantom_2d(d["nx"], d["nx"], d["n_shapes"], d["phantom_seed"]).ravel()
    y = add_gaussian_noise_snr(p.A @ x_true, d["snr_db"], d["noise_seed"])
    x_lsq = np.linalg.lstsq(p.A.toarray(), y, rcond=None)[0] if name == "e1" else None
    return p, y, x_true, x_lsq, lipschitz(p.A)


def oracle_ds_curve(p, y, x_lsq, R, B, mu, n_products, n_points=8, seed=1, **kw):
    """The oracle's DS = ||x - x_lsq|| at n_points equally spaced iteration counts, as
    (products, DS) pairs; 2 R B products per iteration."""
    from oracle.bsgd import ds, run
    per = 2 * R * B
    iters = max(n_products // per, n_points)
    marks = {round(iters * (i + 1) / n_points) for i in range(n_points)}
    out = []
    run(p, y, mu, R, B, iters, seed=seed, callback=lambda st: out.append((st.k * per, ds(st.x, x_lsq)))
        if st.k in marks else None, **kw)
    return out
