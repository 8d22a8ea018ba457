"""The boundary's options against the oracle or the plain path: projected-area sampling
(Algorithm 2, Sec. II-A) with the library's area table, the allocator hook (PyTorch's
caching allocator) and the asynchronous stopping statistic."""
import math

import numpy as np
import pytest

from bsgd_inputs.configs import GeometrySpec
from oracle.area import area_weights
from oracle.bsgd import quantise, run

from helpers import SMALL, log, oracle_matrix, oracle_problem, rel_l2, require_gpu
from test_gpu_solver import _data, _mu, _check_schedule

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["fan", "cone", "parallel"])
def test_area_table_matches_oracle(name):
    from paper_1903_11874_amd import Geometry
    require_gpu()
    g = SMALL[name].with_(im_mode="area", su=SMALL[name].su if name != "parallel" else 3)
    log(f"area table {name}")
    geom = Geometry(g)
    w_lib = geom.table("im_area")
    w_ref = area_weights(g)
    assert np.allclose(w_lib, w_ref, rtol=1e-9, atol=1e-9)
    q_lib = geom.table("im_table").astype(np.int64)
    q_ref = quantise(w_ref).astype(np.int64)
    assert np.max(np.abs(q_lib - q_ref)) <= 1
    assert np.count_nonzero(q_lib) > 0


@pytest.mark.parametrize("name,R,B", [("fan", 1, 3), ("cone", 1, 4)])
def test_trajectory_area_sampled(name, R, B):
    """BSGD-IM with the projected-area weights: draws bit for bit and iterates within
    1e-5 of the oracle fed the library's table."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    log(f"trajectory area-sampled {name}")
    g = SMALL[name].with_(im_mode="area")
    base = g.with_(im_mode="none")
    p = oracle_problem(base)
    A, x_true, y64, y32 = _data(base, 3)
    geom = Geometry(g)
    q = geom.table("im_table")
    mu = _mu(A, 0.3)
    trace = []
    st = run(p, y64, mu, R, B, 40, 11, q=q, trace=trace)
    x = torch.zeros(A.shape[1], device=dev)
    s = Solver(geom, torch.tensor(y32, device=dev), x, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=11)
    s.step(40)
    torch.cuda.synchronize()
    _check_schedule(p, trace, s)
    assert rel_l2(x.double().cpu().numpy(), st.x) <= 1e-5


def test_torch_allocator_gives_the_same_iterates():
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    log("torch allocator")
    g = SMALL["cone"]
    A, x_true, y64, y32 = _data(g, 3)
    mu = _mu(A, 0.3)
    yd = torch.tensor(y32, device=dev)
    xs = [torch.zeros(A.shape[1], device=dev) for _ in range(2)]
    torch.cuda.synchronize()
    used0 = torch.cuda.memory_allocated()
    geom_t = Geometry(g, allocator="torch")
    used_geom = torch.cuda.memory_allocated()
    assert used_geom > used0  # the geometry's tables came from the caching allocator
    for geom, x in zip((Geometry(g), geom_t), xs):
        s = Solver(geom, yd, x, rows_per_iter=1, blocks_per_iter=4, mu=mu, seed=5, tv_lambda=0.2)
        if geom is geom_t:
            assert torch.cuda.memory_allocated() > used_geom  # and the solver state
        s.step(3 * s.epoch_iters)
        torch.cuda.synchronize()
        s.close()
    assert torch.equal(xs[0], xs[1])
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == used_geom  # the solver gave its state back
    geom_t.close()
    assert torch.cuda.memory_allocated() == used0


def test_async_normal_residual_equals_synchronous():
    import torch
    from paper_1903_11874_amd import Geometry, Solver, normal_residual
    from paper_1903_11874_amd.bsgd import normal_residual_async
    dev = require_gpu()
    log("async normal residual")
    solvers, xs = [], []
    for name, seed in (("fan", 3), ("parallel", 4)):
        g = SMALL[name]
        A, x_true, y64, y32 = _data(g, seed)
        geom = Geometry(g)
        x = torch.zeros(A.shape[1], device=dev)
        s = Solver(geom, torch.tensor(y32, device=dev), x, rows_per_iter=1, blocks_per_iter=2,
                   mu=_mu(A, 0.3), seed=seed)
        s.step(7)
        solvers.append(s)
    ref = normal_residual(solvers, relative=True)
    out = torch.zeros(2 * len(solvers), dtype=torch.float64, pin_memory=True)
    for rep in range(2):
        normal_residual_async(solvers, out)
        torch.cuda.current_stream().synchronize()
        got = np.sqrt(out[0::2].numpy()) / np.sqrt(out[1::2].numpy())
        assert np.array_equal(got, ref), (rep, got, ref)
