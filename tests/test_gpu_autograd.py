"""torch.autograd through the HIP projector: gradient vs the FP64 oracle and vs central
finite differences; the scaled-up cone case runs and keeps the adjoint identity."""
import numpy as np
import pytest

from bsgd_inputs.configs import workload
from bsgd_inputs.phantoms import phantom_for, random_image, add_gaussian_noise
from oracle.cfast import Projector
from oracle import tv as otv

from helpers import SMALL, log, oracle_matrix, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _tv_grad_smooth(x, eps):
    """Gradient of sum sqrt(|D x|^2 + eps) (backward differences), FP64 numpy."""
    d = otv.grad(x)
    n = np.sqrt(np.sum(d * d, axis=0) + eps)
    return otv.grad_adjoint(d / n[None])


def test_gradient_matches_oracle_small_cone():
    import torch
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.autograd import project, tv_smooth
    dev = require_gpu()
    g = SMALL["cone"]
    log("autograd small cone")
    A = oracle_matrix(g)
    geom = Geometry(g)
    x0 = random_image(A.shape[1], 5)
    y = random_image(A.shape[0], 6, 0.0, 4.0)
    x = torch.tensor(x0, dtype=torch.float32, device=dev, requires_grad=True)
    yd = torch.tensor(y, dtype=torch.float32, device=dev)
    shape = (g.nz, g.ny, g.nx)
    lam, eps = 1e-3, 1e-8
    loss = 0.5 * ((project(x, geom) - yd).double() ** 2).sum() + lam * tv_smooth(x, shape, eps).double()
    loss.backward()
    gx = x.grad.double().cpu().numpy()
    x32 = x.detach().double().cpu().numpy()
    ref = A.T @ (A @ x32 - yd.double().cpu().numpy()) + lam * _tv_grad_smooth(x32.reshape(shape), eps).ravel()
    assert rel_l2(gx, ref) <= 1e-5


def test_finite_differences_c5():
    """128^3 cone, 180 views of 192^2: loss 1/2||y - A x||^2 + 1e-3 TV(x); central
    differences (eps 1e-3) along 64 seeded random directions."""
    import torch
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.autograd import project, tv_smooth
    dev = require_gpu()
    wl = workload("c5_cone128")
    g = wl.geometry
    log("autograd c5 finite differences")
    geom = Geometry(g)
    x_true = torch.tensor(phantom_for(g, wl.n_shapes, wl.phantom_seed), dtype=torch.float32, device=dev)
    y = geom.forward_project(x_true)
    yd = torch.tensor(add_gaussian_noise(y.double().cpu().numpy(), 0.01, wl.noise_seed), dtype=torch.float32,
                      device=dev)
    shape = (g.nz, g.ny, g.nx)

    def loss_of(xv):
        return 0.5 * ((project(xv, geom) - yd).double() ** 2).sum() + 1e-3 * tv_smooth(xv, shape, 1e-6).double()

    x = (0.5 * x_true).clone().requires_grad_(True)
    loss_of(x).backward()
    grad = x.grad.detach()
    rng = np.random.Generator(np.random.PCG64(3005))
    fd, an = [], []
    with torch.no_grad():
        for _ in range(64):
            d = torch.tensor(rng.normal(size=x.numel()), dtype=torch.float32, device=dev)
            lp = float(loss_of(x.detach() + 1e-3 * d))
            lm = float(loss_of(x.detach() - 1e-3 * d))
            fd.append((lp - lm) / 2e-3)
            an.append(float(torch.dot(grad.double(), d.double())))
    assert rel_l2(np.array(an), np.array(fd)) <= 2e-3
    # the data-term gradient against the FP64 matrix-free oracle
    P = Projector(g)
    xh = x.detach().double().cpu().numpy()
    ref = P.bp(P.fp(xh) - yd.double().cpu().numpy())
    xg = x.detach().clone().requires_grad_(True)
    (0.5 * ((project(xg, geom) - yd).double() ** 2).sum()).backward()
    assert rel_l2(xg.grad.double().cpu().numpy(), ref) <= 1e-5


def test_scaled_cone_512():
    """512^3 volume, 720 views of a 1024^2 detector: one forward and backward pass;
    sampled rays against the oracle and the adjoint identity."""
    import torch
    from bsgd_inputs.configs import GeometrySpec
    from paper_1903_11874_amd import Geometry
    from paper_1903_11874_amd.autograd import project
    dev = require_gpu()
    base = workload("c5_cone128").geometry
    g = base.with_(nx=512, ny=512, nz=512, vx=0.25, vy=0.25, vz=0.25, n_views=720, nu=1024, nv=1024,
                   du=0.5, dv=0.5, bx=4, by=4, bz=4)
    log("autograd 512^3 / 720 x 1024^2")
    geom = Geometry(g)
    x = torch.tensor(phantom_for(g.with_(nx=64, ny=64, nz=64), 8, 7).reshape(64, 64, 64), dtype=torch.float32,
                     device=dev)
    x = torch.nn.functional.interpolate(x[None, None], size=(512, 512, 512), mode="nearest")[0, 0].reshape(-1)
    x = x.contiguous().requires_grad_(True)
    ax = project(x, geom)
    r = torch.tensor(random_image(ax.numel(), 8, -1.0, 1.0), dtype=torch.float32, device=dev)
    (ax * r).sum().backward()
    atr = x.grad.detach()
    lhs = float(torch.dot(ax.detach().double(), r.double()))
    rhs = float(torch.dot(x.detach().double(), atr.double()))
    assert abs(lhs - rhs) <= 1e-6 * float(torch.linalg.norm(ax.detach().double()) * torch.linalg.norm(r.double()))
    sample = np.sort(np.random.Generator(np.random.PCG64(2)).choice(ax.numel(), 400, replace=False))
    ref = Projector(g, rays=sample).fp(x.detach().double().cpu().numpy())
    assert rel_l2(ax.detach().double().cpu().numpy()[sample], ref) <= 1e-5
