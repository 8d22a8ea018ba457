"""Edge and degenerate cases of the HIP path against the oracle: empty view lists, a
step length of zero, zero data, one view and one block, one-pixel blocks, and inputs
the library must refuse. (Rays that miss the image, ragged tiles and blocks smaller than
a workgroup tile occur in every small parity geometry.)"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle.bsgd import run, lipschitz
from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise

from helpers import SMALL, log, oracle_matrix, oracle_problem, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _data(g, seed=5):
    A = oracle_matrix(g)
    x_true = phantom_for(g, 4, seed)
    y32 = add_gaussian_noise(A @ x_true, 0.01, seed + 100).astype(np.float32)
    return A, y32.astype(np.float64), y32


def _trajectory(g, n_iter, R, B, seed, mu_scale=0.3, data=None):
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    A, y64, y32 = data if data is not None else _data(g)
    mu = float(np.float32(mu_scale / (2.0 * lipschitz(A)))) if mu_scale else 0.0
    st = run(oracle_problem(g), y64, mu, R, B, n_iter, seed)
    geom = Geometry(g)
    x = torch.zeros(A.shape[1], dtype=torch.float32, device=dev)
    s = Solver(geom, torch.tensor(y32, device=dev), x, rows_per_iter=R, blocks_per_iter=B, mu=mu, seed=seed)
    s.step(n_iter)
    torch.cuda.synchronize()
    return st, s, x


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_empty_view_list(name):
    """No views: the forward projection returns an empty result, the back projection
    sets the block's voxels to 0 (and adds nothing when accumulating)."""
    import torch
    from paper_1903_11874_amd import Geometry
    dev = require_gpu()
    log(f"empty view list {name}")
    g = SMALL[name]
    geom = Geometry(g)
    n = g.nx * g.ny * g.nz
    x = torch.rand(n, device=dev)
    y = geom.forward_project(x, views=[])
    assert y.numel() == 0
    xb = torch.full((n,), 3.0, device=dev)
    geom.back_project(y, views=[], out=xb, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(xb == 3.0)
    geom.back_project(y, views=[], block=1, out=xb)
    torch.cuda.synchronize()
    from oracle.geometry import column_blocks
    inside = np.zeros(n, dtype=bool)
    inside[column_blocks(g)[1]] = True
    out = xb.cpu().numpy()
    assert np.all(out[inside] == 0.0) and np.all(out[~inside] == 3.0)


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_zero_step_length_keeps_the_image_and_builds_the_memories(name):
    """mu = 0: x never moves, and after a whole epoch g is the sum of the row-block
    gradient memories 2 A_i^T (y - sum_j z^j) the oracle builds."""
    import torch
    log(f"mu = 0 {name}")
    g = SMALL[name]
    st, s, x = _trajectory(g, 2 * g.n_row_blocks * g.n_blocks, 1, 1, seed=9, mu_scale=0.0)
    assert torch.count_nonzero(x).item() == 0
    gsum = s.state("g").double().cpu().numpy()
    assert np.linalg.norm(st.gsum) > 0
    assert rel_l2(gsum, st.gsum) <= TOL


@pytest.mark.parametrize("name", ["parallel", "cone"])
def test_zero_data_stays_zero(name):
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    dev = require_gpu()
    log(f"zero data {name}")
    g = SMALL[name]
    n = g.nx * g.ny * g.nz
    geom = Geometry(g)
    y = torch.zeros(g.n_views * g.nv * g.nu, device=dev)
    x = torch.zeros(n, device=dev)
    s = Solver(geom, y, x, rows_per_iter=1, blocks_per_iter=2, mu=1e-3, seed=1, tv_lambda=0.5)
    rn = s.step(3 * g.n_row_blocks * g.n_blocks, residual=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0 and rn == 0.0


@pytest.mark.parametrize("name,patch", [
    # one view, one row block and one column block: Algorithm 1 is gradient descent
    ("fan", dict(n_views=1, n_row_blocks=1, bx=1, by=1, su=1)),
    ("cone", dict(n_views=1, n_row_blocks=1, bx=1, by=1, bz=1, su=1, sv=1)),
    # one-pixel blocks (one column block per pixel) on a small image
    ("parallel", dict(nx=7, ny=5, nu=12, bx=7, by=5, n_views=9, n_row_blocks=3)),
])
def test_degenerate_partitions(name, patch):
    log(f"degenerate partition {name} {patch}")
    g = SMALL[name].with_(**patch)
    R, B = 1, max(1, g.n_blocks // 3)
    st, s, x = _trajectory(g, 3 * g.n_row_blocks * g.n_blocks // (R * B) + 1, R, B, seed=4)
    assert rel_l2(x.double().cpu().numpy(), st.x) <= TOL


def test_invalid_inputs_are_refused():
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    from paper_1903_11874_amd.bsgd import BsgdError
    dev = require_gpu()
    log("refused inputs")
    g = SMALL["fan"]
    geom = Geometry(g)
    n = g.nx * g.ny
    x = torch.zeros(n, device=dev)
    with pytest.raises(BsgdError):
        geom.forward_project(x, views=[g.n_views])          # view out of range
    with pytest.raises(BsgdError):
        geom.forward_project(x, block=g.n_blocks)           # block out of range
    with pytest.raises(BsgdError):
        geom.back_project(torch.zeros(g.n_views * g.nu, device=dev), scale=math.inf)
    y = torch.zeros(g.n_views * g.nu, device=dev)
    with pytest.raises(BsgdError):
        Solver(geom, y, x, rows_per_iter=g.n_row_blocks + 1, blocks_per_iter=1, mu=1e-3)
    with pytest.raises(BsgdError):
        Solver(geom, y, x, rows_per_iter=1, blocks_per_iter=g.n_blocks + 1, mu=1e-3)
    with pytest.raises(BsgdError):
        geom.set_tuning(fp_views_per_group=0)


@pytest.mark.parametrize("name", ["fan", "cone"])
def test_divergence_is_reported(name):
    """A step length far beyond 1 / (2 ||A||^2) makes the iterates overflow: the residual
    norm is not finite and bsgd_step reports BSGD_E_DIVERGED (status 5); the solver stays
    usable, so a further step with a residual still reports it."""
    import torch
    from paper_1903_11874_amd import Geometry, Solver
    from paper_1903_11874_amd.bsgd import BsgdError
    dev = require_gpu()
    log(f"divergence {name}")
    g = SMALL[name]
    A, y64, y32 = _data(g)
    mu = float(1e10 / (2.0 * lipschitz(A)))  # a growth of about 1e10 per effective epoch
    x = torch.zeros(A.shape[1], device=dev)
    s = Solver(Geometry(g), torch.tensor(y32, device=dev), x, rows_per_iter=1, blocks_per_iter=2, mu=mu, seed=2,
               eager=True)
    with pytest.raises(BsgdError) as e:
        s.step(300, residual=True)
    assert e.value.status == 5
    assert not bool(torch.isfinite(x).all())
    with pytest.raises(BsgdError) as e:
        s.step(1, residual=True)
    assert e.value.status == 5
