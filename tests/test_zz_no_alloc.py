"""The allocation-free normal residual (static device scratch) against the allocating
entry point it varies, through the C ABI: two calls in a row, the second on a smaller
geometry, and the size limit refused before any device work."""
from __future__ import annotations

import math

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec
from tests.helpers import log, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

BIG = GeometrySpec(kind="fan2d", nx=160, ny=144, nz=1, vx=0.5, vy=0.5, vz=0.5, n_views=120,
                   angle_span=2 * math.pi, nu=200, nv=1, du=1.0, dv=1.0, sod=200.0, sdd=400.0,
                   bx=4, by=3, bz=1, n_row_blocks=6, partition_seed=71)
SMALL = GeometrySpec(kind="cone3d", nx=20, ny=18, nz=14, vx=1.0, vy=1.0, vz=0.947, n_views=24,
                     angle_span=2 * math.pi, nu=28, nv=22, du=1.3, dv=1.2373, sod=40.0, sdd=90.0,
                     bx=2, by=3, bz=2, n_row_blocks=4, partition_seed=23)
# 4096^2 voxels alone need 64 MiB of scratch: over the limit
TOO_BIG = GeometrySpec(kind="fan2d", nx=4096, ny=4096, nz=1, vx=0.05, vy=0.05, vz=0.05, n_views=4,
                       angle_span=2 * math.pi, nu=16, nv=1, du=20.0, dv=1.0, sod=400.0, sdd=800.0,
                       bx=4, by=4, bz=1, n_row_blocks=1, partition_seed=72)


def _case(spec, seed, dev):
    import torch
    from paper_1903_11874_amd import Geometry
    rng = np.random.default_rng(seed)
    geom = Geometry(spec)
    n_vox = spec.nx * spec.ny * spec.nz
    n_rays = spec.n_views * spec.nu * spec.nv
    x = torch.tensor(rng.uniform(0.0, 1.0, n_vox), dtype=torch.float32, device=dev)
    y = torch.tensor(rng.uniform(0.0, 5.0, n_rays), dtype=torch.float32, device=dev)
    return geom, x, y


def _allocating(geom, x, y):
    import torch
    from paper_1903_11874_amd import Solver, normal_residual
    xs = x.clone()
    s = Solver(geom, y, xs, rows_per_iter=1, blocks_per_iter=1, mu=0.0, seed=1)
    out = float(normal_residual([s], relative=False)[0])
    torch.cuda.synchronize()
    s.close()
    return out


def test_noalloc_normal_residual_matches_allocating_entry_point():
    dev = require_gpu()
    from paper_1903_11874_amd.bsgd import normal_residual_noalloc, noalloc_scratch_bytes
    assert noalloc_scratch_bytes() == 64 << 20
    for spec, seed in ((BIG, 5), (SMALL, 6)):
        log(f"no-alloc normal residual {spec.kind} {spec.nx}x{spec.ny}x{spec.nz}, {spec.n_views} views")
        geom, x, y = _case(spec, seed, dev)
        ref = _allocating(geom, x, y)
        got = normal_residual_noalloc(geom, y, x)
        assert ref > 0 and math.isfinite(got)
        assert rel_l2([got], [ref]) <= 1e-5, (got, ref)
        # the static scratch keeps the last call's contents: a repeat gives the same value
        assert normal_residual_noalloc(geom, y, x) == got


def test_noalloc_refuses_geometries_over_the_scratch_limit():
    dev = require_gpu()
    from paper_1903_11874_amd import BsgdError
    from paper_1903_11874_amd.bsgd import normal_residual_noalloc
    log("no-alloc size limit (4096^2 fan)")
    geom, x, y = _case(TOO_BIG, 7, dev)
    with pytest.raises(BsgdError, match="E_INVALID_ARG"):
        normal_residual_noalloc(geom, y, x)
