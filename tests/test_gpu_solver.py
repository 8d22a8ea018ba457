"""GPU BSGD iterates against the FP64 oracle: same seeds, same inputs.

Selections (row blocks, column blocks) and importance-sampling draws must match
bit for bit; images must match within 1e-5 relative l2.
"""
import numpy as np
import pytest

from bsgd_inputs.configs import workload
from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise
from oracle.bsgd import run, lipschitz, im_table, tv_period

from helpers import SMALL, log, oracle_matrix, oracle_problem, rel_l2, require_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _data(g, seed=3):
    A = oracle_matrix(g)
    x_true = phantom_for(g, 6, seed)
    y = add_gaussian_noise(A @ x_true, 0.01, seed + 100)
    y32 = y.astype(np.float32)
    return A, x_true, y32.astype(np.float64), y32


def _mu(A, scale):
    return float(np.float32(scale / (2.0 * lipschitz(A))))


def _pair(g, n_iter, R, B, seed, im=None, tv_lambda=0.0, mu_scale=0.3, data_seed=3, im_until=0, subdet=False,
          eager=False, bp_waves=None):
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    p = oracle_problem(g)
    A, x_true, y64, y32 = _data(g, data_seed)
    mu = _mu(A, mu_scale)
    q = im_table(p, im) if im else None
    trace = []
    st = run(p, y64, mu, R, B, n_iter, seed, q=q, tv_lambda=tv_lambda, trace=trace, im_until=im_until or None,
             subdet_memory=subdet)
    geom = Geometry(g.with_(im_mode=im or "none"), im_table=q)
    if bp_waves is not None:
        geom.set_tuning(bp_waves=bp_waves)
        assert geom.bp_waves == bp_waves
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], dtype=torch.float32, device=dev)
    solver = Solver(geom, yd, xd, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=seed, tv_lambda=tv_lambda,
                    tv_inner_iters=20, im_until=im_until, subdet_memory=subdet, eager=eager)
    rn = solver.step(n_iter, residual=True)
    return p, st, trace, solver, xd, rn


def _check_schedule(p, trace, solver, tail_from=None):
    rows, blocks, draws = solver.last_schedule()
    assert rows.shape[0] == len(trace)
    for it, t in enumerate(trace):
        assert list(rows[it]) == t["rows"], it
        assert list(blocks[it]) == t["blocks"], it
        if tail_from is not None and it >= tail_from:
            n_views = sum(len(p.groups[i]) for i in t["rows"])
            assert np.all(draws[it, :n_views, :] == -2), it  # every ray, no sampling
        elif t["draws"]:
            views = [v for i in t["rows"] for v in p.groups[i]]
            for a, v in enumerate(views):
                for b, j in enumerate(t["blocks"]):
                    assert int(draws[it, a, b]) == t["draws"][(v, j)], (it, v, j)


@pytest.mark.parametrize("name,R,B", [("fan", 1, 2), ("parallel", 2, 3), ("cone", 1, 4), ("fan_wide", 1, 2),
                                      ("cone_wide", 2, 3)])
def test_trajectory_plain(name, R, B):
    log(f"trajectory plain {name} R={R} B={B}")
    p, st, trace, solver, xd, rn = _pair(SMALL[name], 60, R, B, seed=7)
    _check_schedule(p, trace, solver)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


@pytest.mark.parametrize("name,waves,im", [("fan", 2, "colnorm"), ("fan", 8, "colnorm"), ("parallel", 8, None),
                                           ("fan_wide", 2, None)])
def test_trajectory_back_projection_waves(name, waves, im):
    """Every wave split of the 2D back projector (a tuned launch shape: the views of a
    voxel gathered by that many waves, their sums added in a fixed order) follows the
    oracle, on the LDS-staged and the global-memory forward paths."""
    log(f"trajectory 2D back projection over {waves} waves {name}")
    p, st, trace, solver, xd, rn = _pair(SMALL[name], 40, 2, 3, seed=17, im=im, bp_waves=waves)
    _check_schedule(p, trace, solver)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_trajectory_importance_sampled_unbiased_tail(name):
    """Importance sampling for the first 20 iterations, every ray afterwards (the
    unbiased tail): same iterates and draws as the oracle."""
    log(f"trajectory IM + unbiased tail {name}")
    p, st, trace, solver, xd, rn = _pair(SMALL[name], 45, 2, 3, seed=13, im="colnorm", im_until=20)
    _check_schedule(p, trace, solver, tail_from=20)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


@pytest.mark.parametrize("name,R,B,im", [("fan", 2, 3, "colnorm"), ("cone", 1, 4, "colnorm"),
                                         ("cone", 2, 2, "uniform")])
def test_trajectory_importance_sampled(name, R, B, im):
    log(f"trajectory IM {name} {im}")
    p, st, trace, solver, xd, rn = _pair(SMALL[name], 50, R, B, seed=11, im=im)
    _check_schedule(p, trace, solver)
    assert any(s >= 0 for t in trace for s in t["draws"].values())
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL


@pytest.mark.parametrize("name,R,B,im,tv", [("fan", 2, 3, "colnorm", 0.0), ("cone", 1, 4, "colnorm", 0.0),
                                            ("cone", 2, 2, "uniform", 0.0), ("parallel", 1, 2, None, 0.5),
                                            ("fan_wide", 1, 2, None, 0.0)])
def test_trajectory_subdetector_memory(name, R, B, im, tv):
    """Gradient memory per (view, sub-detector, block): same iterates, g and residual
    norm as the oracle's per-part memories, over whole graph-replayed epochs."""
    g = SMALL[name]
    log(f"trajectory sub-detector memory {name} R={R} B={B} im={im} tv={tv}")
    n = 2 * tv_period(g.n_row_blocks, g.n_blocks, R, B) + 5
    p, st, trace, solver, xd, rn = _pair(g, n, R, B, seed=17, im=im, tv_lambda=tv, subdet=True)
    _check_schedule(p, trace, solver)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert rel_l2(solver.state("g").double().cpu().numpy(), st.gsum) <= 1e-4
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)
    rho = solver.state("rho")
    assert rho.numel() == solver.geom.info["z_floats"] and bool(rho.abs().sum() > 0)


def test_subdetector_memory_graphs_equal_eager_and_batch_refuses_it():
    import torch
    from paper_1903_11874_amd import Geometry, Solver, step_batch
    from paper_1903_11874_amd.bsgd import BsgdError
    g = SMALL["fan"]
    T = tv_period(g.n_row_blocks, g.n_blocks, 1, 3)
    log("sub-detector memory: graphs vs eager")
    xs = []
    for eager in (False, True):
        _, _, _, solver, xd, _ = _pair(g, 3 * T, 1, 3, seed=19, im="colnorm", subdet=True, eager=eager)
        xs.append(xd.cpu().numpy())
        with pytest.raises(BsgdError):
            solver.state("ghat")
        with pytest.raises(BsgdError):
            step_batch([solver], 1)
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("name", ["parallel", "cone"])
def test_trajectory_tv(name):
    g = SMALL[name]
    T = tv_period(g.n_row_blocks, g.n_blocks, 1, 2)
    log(f"trajectory TV {name} T={T}")
    p, st, trace, solver, xd, rn = _pair(g, 2 * T + 3, 1, 2, seed=5, tv_lambda=0.5)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL


def test_all_blocks_is_gradient_descent():
    g = SMALL["fan"]
    log("GD special case")
    p, st, trace, solver, xd, rn = _pair(g, 30, g.n_row_blocks, g.n_blocks, seed=1, mu_scale=0.4)
    A = p.A
    y = st.r + st.z.sum(axis=0)  # the y the oracle used
    x = np.zeros(A.shape[1])
    mu = _mu(A, 0.4)
    for _ in range(30):
        x = x + 2 * mu * (A.T @ (y - A @ x))
    assert rel_l2(xd.double().cpu().numpy(), x) <= TOL


def test_c1_configuration():
    """The small workload in full: 2D parallel 64x64, 90 views, 9 row blocks, 16 blocks,
    one (row, column) pair per iteration, 20 effective epochs (2880 iterations)."""
    wl = workload("c1_parallel64")
    g = wl.geometry
    T = tv_period(g.n_row_blocks, g.n_blocks, 1, 1)
    n = wl.solver.effective_epochs * T
    log(f"C1 full run {n} iterations")
    p, st, trace, solver, xd, rn = _pair(g, n, 1, 1, seed=wl.solver.seed, mu_scale=0.5,
                                         data_seed=wl.phantom_seed)
    _check_schedule(p, trace, solver)
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
    assert abs(rn - np.linalg.norm(st.r)) <= TOL * np.linalg.norm(st.r)


def test_state_invariants_and_determinism():
    import torch
    g = SMALL["fan"]
    log("invariants")
    p, st, trace, solver, xd, rn = _pair(g, 40, 2, 3, seed=13, im="colnorm")
    ghat = solver.state("ghat").view(g.n_row_blocks, -1).double()
    gsum = solver.state("g").double()
    assert rel_l2(gsum.cpu().numpy(), ghat.sum(0).cpu().numpy()) <= TOL
    assert rel_l2(gsum.cpu().numpy(), st.gsum) <= TOL
    _, _, _, solver2, xd2, rn2 = _pair(g, 40, 2, 3, seed=13, im="colnorm")
    assert torch.equal(xd, xd2) and rn == rn2


def test_node_count_rule_and_errors():
    import torch
    from paper_1903_11874_amd import Geometry, Solver, BsgdError
    dev = require_gpu()
    g = SMALL["fan"]  # M = 5, N = 9
    geom = Geometry(g)
    y = torch.zeros(g.n_views * g.nu, device=dev)
    x = torch.zeros(g.nx * g.ny, device=dev)
    s = Solver(geom, y, x, node_count=3, mu=1e-4, seed=1)
    assert (s.rows_per_iter, s.blocks_per_iter) == (1, 3)
    s = Solver(geom, y, x, node_count=18, mu=1e-4, seed=1)
    assert (s.rows_per_iter, s.blocks_per_iter) == (2, 9)
    for bad in (dict(node_count=10), dict(rows_per_iter=6, blocks_per_iter=1), dict(rows_per_iter=1),
                dict(node_count=3, im_until=-1)):
        with pytest.raises(BsgdError) as e:
            Solver(geom, y, x, mu=1e-4, **bad)
        assert e.value.status == 1
    # an unknown flag bit is rejected before any device work
    s = Solver(geom, y, x, node_count=3, mu=1e-4, seed=1)
    s.options.flags = 4
    from paper_1903_11874_amd.bsgd import load_library, _dev_ptr, _stream_ptr
    import ctypes
    h = ctypes.c_void_p()
    st = load_library().bsgd_solver_create(geom.handle, _dev_ptr(y), _dev_ptr(x), ctypes.byref(s.options),
                                           _stream_ptr(None), ctypes.byref(h))
    assert st == 1 and h.value is None


def test_solve_matches_stepping():
    import torch
    from paper_1903_11874_amd import Geometry, Solver, solve
    dev = require_gpu()
    g = SMALL["parallel"]
    log("solve api")
    A, x_true, y64, y32 = _data(g)
    mu = _mu(A, 0.3)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    x1 = torch.zeros(A.shape[1], device=dev)
    it, rn = solve(geom, yd, x1, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=4, max_effective_epochs=3)
    x2 = torch.zeros(A.shape[1], device=dev)
    s = Solver(geom, yd, x2, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=4)
    s.step(3 * s.epoch_iters)
    assert it == 3 * s.epoch_iters and torch.equal(x1, x2)
    # with a tolerance the solve stops early once ||A^T(y - Ax)|| / ||A^T y|| <= tol
    x3 = torch.zeros(A.shape[1], device=dev)
    it3, _ = solve(geom, yd, x3, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=4, max_effective_epochs=200,
                   tol=0.05)
    x3n = x3.double().cpu().numpy()
    ratio = np.linalg.norm(A.T @ (y64 - A @ x3n)) / np.linalg.norm(A.T @ y64)
    assert it3 < 200 * s.epoch_iters and ratio <= 0.05 * 1.001


@pytest.mark.parametrize("name,im,tv", [("fan", "colnorm", 0.0), ("cone", None, 0.5), ("parallel", None, 0.0)])
def test_graph_replay_matches_eager(name, im, tv):
    """Whole-epoch calls replay a captured HIP graph; every replay must equal the eager
    launches bit for bit, with other device work and synchronisations in between."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = SMALL[name].with_(im_mode=im or "none")
    log(f"graph replay {name} im={im} tv={tv}")
    A, x_true, y64, y32 = _data(SMALL[name])
    mu = _mu(A, 0.3)
    p = oracle_problem(SMALL[name])
    geom = Geometry(g, im_table=im_table(p, im) if im else None)
    yd = torch.tensor(y32, device=dev)
    xg = torch.zeros(A.shape[1], device=dev)
    xe = torch.zeros(A.shape[1], device=dev)
    sg = Solver(geom, yd, xg, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=21, tv_lambda=tv)
    se = Solver(geom, yd, xe, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=21, tv_lambda=tv, eager=True)
    T = sg.epoch_iters
    for rep in range(4):
        sg.step(T if rep % 2 == 0 else 2 * T)
        se.step(T if rep % 2 == 0 else 2 * T)
        junk = geom.forward_project(xg)  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), rep
        assert float(junk.sum()) == float(junk.sum())
    rg, bg, dg = sg.last_schedule()
    re_, be, de = se.last_schedule()
    assert np.array_equal(rg, re_) and np.array_equal(bg, be) and np.array_equal(dg, de)
    # a call that does not start at an epoch boundary runs eagerly and stays in step
    sg.step(3)
    se.step(3)
    sg.step(T)
    se.step(T)
    torch.cuda.synchronize()
    assert torch.equal(xg, xe)


def test_batched_graphs_equal_solo_solves():
    """Whole-epoch batched calls of a recurring set of solves are captured once and
    replayed as HIP graphs; every replay equals the solves run alone, bit for bit, with
    unrelated device work and synchronisations between replays, and a new subset gets
    its own graph."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver, step_batch
    dev = require_gpu()
    log("batched graphs vs solo")
    g = SMALL["fan"]
    A, x_true, y64, y32 = _data(g, 41)
    mu = _mu(A, 0.3)
    p = oracle_problem(g)
    geoms = {"none": Geometry(g), "colnorm": Geometry(g.with_(im_mode="colnorm"), im_table=im_table(p, "colnorm"))}
    yd = torch.tensor(y32, device=dev)
    cfg = [("none", 1, 3, 41), ("none", 3, 1, 42), ("colnorm", 1, 3, 43)]  # every one 15 iterations per epoch
    bat, solo = [], []
    for im, R, B, seed in cfg:
        pair = []
        for eager in (False, True):
            x = torch.zeros(A.shape[1], device=dev)
            pair.append((x, Solver(geoms[im], yd, x, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=seed,
                                   eager=eager)))
        bat.append(pair[0])
        solo.append(pair[1])
    T = bat[0][1].epoch_iters
    assert all(b[1].epoch_iters == T for b in bat)
    sets = [[0, 1, 2]] * 4 + [[0, 2]] * 3 + [[0, 1, 2]]
    for rep, idx in enumerate(sets):
        step_batch([bat[i][1] for i in idx], T)
        for i in idx:
            solo[i][1].step(T)
        junk = geoms["none"].forward_project(bat[1][0])  # unrelated work between replays
        torch.cuda.synchronize()
        assert float(junk.sum()) == float(junk.sum())
        for i in range(3):
            assert torch.equal(bat[i][0], solo[i][0]), (rep, i)
            assert bat[i][1].iterations == solo[i][1].iterations
    rb, bb, db = bat[2][1].last_schedule()
    rs, bs, ds_ = solo[2][1].last_schedule()
    assert np.array_equal(rb, rs) and np.array_equal(bb, bs) and np.array_equal(db, ds_)
    # the first solve against the oracle's run of the same iterations
    st = run(p, y64, mu, 1, 3, bat[0][1].iterations, 41)
    assert rel_l2(bat[0][0].double().cpu().numpy(), st.x) <= TOL


def test_batched_solves_equal_solo_solves():
    """Several solves of different geometries in shared launches give bit-identical
    iterates to the same solves run alone."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver, step_batch
    dev = require_gpu()
    log("batched vs solo")
    specs = [(SMALL["fan"].with_(im_mode="colnorm"), 1, 3, 0.0, 31), (SMALL["parallel"], 2, 2, 0.3, 32),
             (SMALL["fan"], 1, 9, 0.0, 33), (SMALL["parallel"], 1, 1, 0.0, 34)]
    geoms, runs = {}, []
    for g, R, B, tv, seed in specs:
        base = g.with_(im_mode="none")
        A, x_true, y64, y32 = _data(base, seed)
        key = (g.kind, g.im_mode)
        if key not in geoms:
            geoms[key] = Geometry(g)
        yd = torch.tensor(y32, device=dev)
        mu = _mu(A, 0.3)
        pair = []
        for _ in range(2):
            x = torch.zeros(A.shape[1], device=dev)
            pair.append((x, Solver(geoms[key], yd, x, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=seed,
                                   tv_lambda=tv, eager=True)))
        runs.append(pair)
    # the geometries' 2D back projections use different wave splits, so each batched
    # iteration launches one back projection per split
    for geom, w in zip(geoms.values(), (2, 8, 4)):
        geom.set_tuning(bp_waves=w)
    for rep, n in enumerate((7, 1, 12)):
        step_batch([r[0][1] for r in runs], n)
        for r in runs:
            r[1][1].step(n)
        torch.cuda.synchronize()
        for i, r in enumerate(runs):
            assert torch.equal(r[0][0], r[1][0]), (rep, i)
    # a batch of a subset, then the rest, keeps every solve in step with its solo twin
    step_batch([runs[1][0][1], runs[3][0][1]], 5)
    step_batch([runs[0][0][1], runs[2][0][1]], 5)
    for r in runs:
        r[1][1].step(5)
    torch.cuda.synchronize()
    for i, r in enumerate(runs):
        assert torch.equal(r[0][0], r[1][0]), i
        assert r[0][1].iterations == r[1][1].iterations
    # and every batched solve against the oracle's run of the same request (the
    # importance-sampled one with the library's exported sampling table)
    for (g, R, B, tv, seed), r in zip(specs, runs):
        base = g.with_(im_mode="none")
        A, x_true, y64, y32 = _data(base, seed)
        geom = geoms[(g.kind, g.im_mode)]
        q = None
        if g.im_mode != "none":
            q = geom.table("im_table").reshape(g.n_views, g.su * g.sv, g.n_blocks)
        st = run(oracle_problem(base), y64, _mu(A, 0.3), R, B, r[0][1].iterations, seed, q=q, tv_lambda=tv)
        assert rel_l2(r[0][0].double().cpu().numpy(), st.x) <= TOL, (g.kind, R, B)


def test_batched_cone_solves_equal_solo_solves_and_the_oracle():
    """Cone-beam solves in shared launches: one whose blocks are staged in LDS by the
    forward projector and one whose blocks are walked in global memory (two forward
    launch classes in one batch), one of them with TV. Each equals its solo twin bit for
    bit and follows the oracle."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver, step_batch
    dev = require_gpu()
    log("batched cone solves vs solo and oracle")
    specs = [(SMALL["cone"], 1, 4, 0.0, 61), (SMALL["cone_wide"], 2, 2, 0.5, 62), (SMALL["cone"], 2, 3, 0.3, 63)]
    geoms, runs = {}, []
    for g, R, B, tv, seed in specs:
        A, x_true, y64, y32 = _data(g, seed)
        if g.nx not in geoms:
            geoms[g.nx] = Geometry(g)
        yd = torch.tensor(y32, device=dev)
        mu = _mu(A, 0.3)
        pair = []
        for _ in range(2):
            x = torch.zeros(A.shape[1], device=dev)
            pair.append((x, Solver(geoms[g.nx], yd, x, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=seed,
                                   tv_lambda=tv, eager=True)))
        runs.append(pair)
    assert geoms[SMALL["cone"].nx].fp_staged and not geoms[SMALL["cone_wide"].nx].fp_staged
    for rep, n in enumerate((9, 1, 14)):
        step_batch([r[0][1] for r in runs], n)
        for r in runs:
            r[1][1].step(n)
        torch.cuda.synchronize()
        for i, r in enumerate(runs):
            assert torch.equal(r[0][0], r[1][0]), (rep, i)
    for (g, R, B, tv, seed), r in zip(specs, runs):
        A, x_true, y64, y32 = _data(g, seed)
        st = run(oracle_problem(g), y64, _mu(A, 0.3), R, B, r[0][1].iterations, seed, tv_lambda=tv)
        assert rel_l2(r[0][0].double().cpu().numpy(), st.x) <= TOL, (g.nx, R, B, tv)


def test_autotuner_shapes_do_not_change_results():
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    from paper_1903_11874_amd.tuning import autotune
    dev = require_gpu()
    log("autotuner")
    g = SMALL["fan"].with_(im_mode="colnorm")
    A, x_true, y64, y32 = _data(SMALL["fan"])
    mu = _mu(A, 0.3)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    timings = autotune(geom, yd, node_count=9, mu=mu, views=(1, 2, 5, 16), splits=(1, 4), epochs=1)
    assert set(timings) == ({(c, s) for c in (1, 2, 5, 16) for s in (1, 4)} |
                            {("bp_waves", w) for w in (2, 4, 8)})
    assert (geom.fp_views_per_group, geom.fp_ray_split) in timings
    assert ("bp_waves", geom.bp_waves) in timings
    with pytest.raises(Exception):
        geom.set_tuning(bp_waves=3)
    geom.set_tuning(bp_waves=4)
    outs = {}
    for sp in (1, 2, 4):
        for c in (1, 4, 16):
            geom.set_tuning(fp_views_per_group=c, fp_ray_split=sp)
            x = torch.zeros(A.shape[1], device=dev)
            Solver(geom, yd, x, node_count=9, mu=mu, seed=3, eager=True).step(20)
            outs[(c, sp)] = x
    # views per workgroup never changes a bit; the ray split only the FP32 rounding
    for sp in (1, 2, 4):
        assert all(torch.equal(outs[(1, sp)], outs[(c, sp)]) for c in (4, 16))
        assert rel_l2(outs[(1, sp)].double().cpu().numpy(), outs[(1, 1)].double().cpu().numpy()) < 1e-5


@pytest.mark.parametrize("name", ["fan_wide", "cone_wide"])
def test_autotuner_waves_per_pair_of_the_global_walk(name):
    # blocks too large for the LDS stage: the tuner searches waves per (view, block)
    # pair, which only regroups the rays among waves, so every shape gives the same bits
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    from paper_1903_11874_amd.tuning import autotune
    dev = require_gpu()
    log(f"autotuner, global walk {name}")
    g = SMALL[name]
    A, x_true, y64, y32 = _data(g)
    mu = _mu(A, 0.3)
    geom = Geometry(g)
    assert not geom.fp_staged
    yd = torch.tensor(y32, device=dev)
    timings = autotune(geom, yd, node_count=4, mu=mu, waves=(1, 3, 16), bp_waves=(), epochs=1)
    assert set(timings) == {(1,), (3,), (16,)}
    assert (geom.fp_waves_per_pair,) in timings
    outs = []
    for w in (1, 2, 5, 64):
        geom.set_tuning(fp_waves_per_pair=w)
        assert geom.fp_waves_per_pair == w
        x = torch.zeros(A.shape[1], device=dev)
        Solver(geom, yd, x, node_count=4, mu=mu, seed=5, eager=True).step(12)
        outs.append(x)
    assert all(torch.equal(outs[0], o) for o in outs[1:])
    with pytest.raises(Exception):
        geom.set_tuning(fp_waves_per_pair=65)


@pytest.mark.parametrize("scale,eager", [(2.0, True), (0.05, False)])
def test_auto_step_length_matches_oracle(scale, eager):
    """Algorithm 3: the same step-length decisions as the oracle, and the iterate."""
    import torch
    from oracle.bsgd import AutoMu
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = SMALL["fan"]
    log(f"auto mu scale={scale}")
    p = oracle_problem(g)
    A, x_true, y64, y32 = _data(g)
    mu = _mu(A, scale)
    am = AutoMu()
    R, B, n = 1, 9, 16 * g.n_row_blocks  # T = M: checks at every epoch boundary
    st = run(p, y64, mu, R, B, n, 17, auto_mu=am)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], device=dev)
    s = Solver(geom, yd, xd, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=17, auto_mu=True, eager=eager)
    s.step(n)
    mu_now, hist = s.step_length()
    assert len(hist) == len(am.mu_history) == 16
    assert np.allclose(hist, am.mu_history, rtol=1e-12)
    assert hist[-1] != mu  # the rule acted
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_normal_residual_matches_oracle(name):
    """The stopping statistic ||A^T (y - A x)|| (and its ratio to ||A^T y||) of several
    solvers in one call equals the oracle's, each at its own image."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver, normal_residual
    dev = require_gpu()
    g = SMALL[name]
    log(f"normal residual {name}")
    A, x_true, y64, y32 = _data(g)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    rng = np.random.Generator(np.random.PCG64(17))
    xs = [torch.tensor(x_true * s + rng.normal(0, 0.05, x_true.size), dtype=torch.float32, device=dev)
          for s in (0.5, 0.9, 1.0)]
    solvers = [Solver(geom, yd, x, node_count=4, mu=1e-3) for x in xs]
    absolute = normal_residual(solvers, relative=False)
    relative = normal_residual(solvers, relative=True)
    ref_y = np.linalg.norm(A.T @ y64)
    for x, a, r in zip(xs, absolute, relative):
        x64 = x.double().cpu().numpy()
        ref = np.linalg.norm(A.T @ (y64 - A @ x64))
        assert abs(a - ref) <= 1e-4 * ref
        assert abs(r - ref / ref_y) <= 1e-4 * ref / ref_y


@pytest.mark.parametrize("scale", [2.0, 0.05])
def test_auto_step_length_with_tv_on_replayed_graphs(scale):
    """Algorithm 3 with the TV prox of Algorithm 4 on captured, replayed epochs (T = M,
    so every epoch ends with a prox and a step-length check): the prox weight mu lambda
    must follow the step-length changes between replays. Same decisions and iterate as
    the oracle; lambda is set so the prox weight matters (mu0 lambda = 0.05)."""
    import torch
    from oracle.bsgd import AutoMu
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    g = SMALL["fan"]
    log(f"auto mu + TV on graphs, scale={scale}")
    p = oracle_problem(g)
    A, x_true, y64, y32 = _data(g)
    mu = _mu(A, scale)
    lam = 0.05 / mu
    R, B = 1, 9
    assert tv_period(g.n_row_blocks, g.n_blocks, R, B) == g.n_row_blocks
    n = 12 * g.n_row_blocks
    am = AutoMu()
    st = run(p, y64, mu, R, B, n, 23, auto_mu=am, tv_lambda=lam)
    geom = Geometry(g)
    yd = torch.tensor(y32, device=dev)
    xd = torch.zeros(A.shape[1], device=dev)
    s = Solver(geom, yd, xd, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=23, auto_mu=True, tv_lambda=lam,
               tv_inner_iters=20)
    s.step(n)
    mu_now, hist = s.step_length()
    assert np.allclose(hist, am.mu_history, rtol=1e-12)
    assert len(set(hist)) > 1  # the step length changed between replays
    assert rel_l2(xd.double().cpu().numpy(), st.x) <= TOL
