"""Solver parity at the launch shapes the throughput measurement runs.

The fan-beam measurement stages 64x64 image tiles in LDS with 12 views per 1024-thread
forward-projection workgroup, runs full 16x8 back-projection pair tiles and draws one
of 4 sub-detectors per (view, block). The cone-beam measurement walks 64x64x16 blocks
with 15-view row blocks and many waves per (view, block) pair. These tests run the same
kernel shapes on reduced detectors and view counts, where the FP64 oracle still
finishes in seconds, and compare iterates (1e-5 relative l2) and draws (bit for bit).
"""
import math

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec
from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise
from oracle.bsgd import run, lipschitz, im_table, tv_period

from helpers import SMALL, log, oracle_matrix, oracle_problem, rel_l2, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5

# 128^2 fan beam at 0.5 mm cut into 2x2 blocks of 64^2 pixels (the fan workload's tile),
# 232 views in 16 row blocks of 14 or 15 views (one full 12-view chunk and a ragged one
# per row block), 192 bins of 1 mm, SOD 500, SDD 1000, 4 sub-detectors.
FAN_TILES = GeometrySpec(kind="fan2d", nx=128, ny=128, nz=1, vx=0.5, vy=0.5, vz=0.5, n_views=232,
                         angle_span=2 * math.pi, nu=192, nv=1, du=1.0, dv=1.0, sod=500.0, sdd=1000.0,
                         bx=2, by=2, bz=1, n_row_blocks=16, partition_seed=31, su=4, sv=1)
# 128x64x16 cone at 0.5 mm cut into two 64x64x16 blocks (the cone workload's block), 30
# views in 2 row blocks of 15, a 160x24 detector of 1 mm pixels, SOD 600, SDD 1200.
CONE_BLOCKS = GeometrySpec(kind="cone3d", nx=128, ny=64, nz=16, vx=0.5, vy=0.5, vz=0.5, n_views=30,
                           angle_span=2 * math.pi, nu=160, nv=24, du=1.0, dv=1.0, sod=600.0, sdd=1200.0,
                           bx=2, by=1, bz=1, n_row_blocks=2, partition_seed=32, su=2, sv=2)


def _data(g, seed):
    A = oracle_matrix(g)
    x_true = phantom_for(g, 8, seed)
    y32 = add_gaussian_noise(A @ x_true, 0.01, seed + 100).astype(np.float32)
    return A, y32.astype(np.float64), y32


def _check_draws(p, trace, solver):
    rows, blocks, draws = solver.last_schedule()
    assert rows.shape[0] == len(trace)
    for it, t in enumerate(trace):
        assert list(rows[it]) == t["rows"] and list(blocks[it]) == t["blocks"], it
        views = [v for i in t["rows"] for v in p.groups[i]]
        for a, v in enumerate(views):
            for b, j in enumerate(t["blocks"]):
                want = t["draws"][(v, j)] if t["draws"] else -2
                assert int(draws[it, a, b]) == want, (it, v, j)


@pytest.mark.parametrize("split,bp_waves", [(1, 4), (4, 4), (1, 2), (1, 8)])
def test_fan_tiles_importance_sampled(split, bp_waves):
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = FAN_TILES.with_(im_mode="colnorm")
    log(f"bench-shaped fan: 64x64 LDS tiles, 12-view chunks, IM S=4, ray split {split}, BP waves {bp_waves}")
    p = oracle_problem(FAN_TILES)
    A, y64, y32 = _data(FAN_TILES, 41)
    mu = float(np.float32(0.5 / (2.0 * lipschitz(A))))
    q = im_table(p, "colnorm")
    R, B = 1, 4
    n = 2 * tv_period(g.n_row_blocks, g.n_blocks, R, B) + 3
    trace = []
    st = run(p, y64, mu, R, B, n, 51, q=q, trace=trace)
    geom = Geometry(g, im_table=q)
    geom.set_tuning(fp_views_per_group=12, fp_ray_split=split, bp_waves=bp_waves)
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], dtype=torch.float32, device=dev)
    s = Solver(geom, yd, xd, node_count=4, mu=mu, seed=51)
    assert (s.rows_per_iter, s.blocks_per_iter) == (R, B)
    rn = s.step(n, residual=True)
    _check_draws(p, trace, s)
    assert any(v >= 0 for t in trace for v in t["draws"].values())
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


@pytest.mark.parametrize("tv", [0.0, 1.0])
def test_cone_blocks(tv):
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = CONE_BLOCKS
    log(f"bench-shaped cone: 64x64x16 blocks, 15-view row blocks, tv={tv}")
    p = oracle_problem(g)
    A, y64, y32 = _data(g, 42)
    mu = float(np.float32(0.5 / (2.0 * lipschitz(A))))
    lam = tv * 0.01 / mu  # prox weight mu lambda = 0.01 when on
    R, B = 1, 2
    n = 3 * tv_period(g.n_row_blocks, g.n_blocks, R, B) + 1
    trace = []
    st = run(p, y64, mu, R, B, n, 52, trace=trace, tv_lambda=lam)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], dtype=torch.float32, device=dev)
    s = Solver(geom, yd, xd, node_count=2, mu=mu, seed=52, tv_lambda=lam, tv_inner_iters=20)
    rn = s.step(n, residual=True)
    _check_draws(p, trace, s)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)
    # the full projectors at this shape, against the explicit matrix
    xt = torch.tensor(phantom_for(g, 8, 42), dtype=torch.float32, device=dev)
    yfp = geom.forward_project(xt).double().cpu().numpy()
    assert rel_l2(yfp, A @ xt.double().cpu().numpy()) <= TOL
    bp = geom.back_project(torch.tensor(y32, device=dev)).double().cpu().numpy()
    assert rel_l2(bp, A.T @ y64) <= TOL


@pytest.mark.parametrize("mode", ["colnorm", "area"])
def test_cone_blocks_importance_sampled(mode):
    # the global-memory walk over one drawn sub-detector of each pair (its part of the
    # pair's ray order), with both weightings; then the unbiased tail (every ray)
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = CONE_BLOCKS.with_(im_mode=mode)
    log(f"bench-shaped cone: 64x64x16 blocks, IM S=4 ({mode})")
    p = oracle_problem(CONE_BLOCKS)
    A, y64, y32 = _data(CONE_BLOCKS, 43)
    mu = float(np.float32(0.5 / (2.0 * lipschitz(A))))
    q = im_table(p, mode)
    R, B = 1, 2
    n = 3 * tv_period(g.n_row_blocks, g.n_blocks, R, B) + 1
    tail = n - 2
    trace = []
    st = run(p, y64, mu, R, B, n, 53, q=q, trace=trace, im_until=tail)
    geom = Geometry(g, im_table=q)
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], dtype=torch.float32, device=dev)
    s = Solver(geom, yd, xd, node_count=2, mu=mu, seed=53, im_until=tail)
    rn = s.step(n, residual=True)
    _check_draws(p, trace, s)
    assert any(v >= 1 for t in trace for v in t["draws"].values())
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


@pytest.mark.parametrize("name", ["cone_blocks", "fan_wide"])
def test_global_walk_batched_warm_start(name):
    # two solves whose blocks exceed the LDS stage (64x64x16 cone blocks; 131x130-pixel
    # fan blocks) from a nonzero image (the walk's copy of x stored y fastest must be
    # built from it), one with TV: batched epochs (eager, captured, replayed) equal solo
    # solves bit for bit, and both equal the oracle
    import torch
    from paper_1903_11874_amd import Geometry, Solver, step_batch
    dev = require_gpu()
    g = CONE_BLOCKS if name == "cone_blocks" else SMALL["fan_wide"]
    log(f"global walk {name}: batched epochs from a nonzero start")
    p = oracle_problem(g)
    geom = Geometry(g)
    assert not geom.fp_staged
    R, B = 1, 2
    T = tv_period(g.n_row_blocks, g.n_blocks, R, B)
    solves = []
    for seed, tv in ((61, 0.0), (62, 1.0)):
        A, y64, y32 = _data(g, seed)
        mu = float(np.float32(0.5 / (2.0 * lipschitz(A))))
        lam = tv * 0.01 / mu
        x0 = (0.5 * phantom_for(g, 6, seed + 7)).astype(np.float32)
        st = run(p, y64, mu, R, B, 3 * T, seed, x0=x0.astype(np.float64), tv_lambda=lam)
        yd = torch.tensor(y32, device=dev)
        pair = []
        for _ in range(2):
            x = torch.tensor(x0, device=dev)
            pair.append((x, Solver(geom, yd, x, node_count=2, mu=mu, seed=seed, tv_lambda=lam, tv_inner_iters=20)))
        solves.append((pair, st))
    for _ in range(3):
        step_batch([pair[0][1] for pair, _ in solves], T)
    for pair, _ in solves:
        pair[1][1].step(3 * T)
    torch.cuda.synchronize()
    for i, (pair, st) in enumerate(solves):
        assert torch.equal(pair[0][0], pair[1][0]), i
        assert rel_l2(pair[0][0].double().cpu().numpy(), st.x) <= TOL, i
