"""Convergence studies on the HIP path (Sec. III-A to III-D and the TV comparison of Sec. III-E).

The paper measures BSGD by the distance to the least-squares solution,
DS = ||x_rec - x_lsq|| (Sec. III-A), against the number of products of a vector with a
sub-matrix A_I^J or its transpose (Sec. III-B), and by the image SNR against the phantom,
20 log10(||x_true|| / ||x_true - x||), for the TV comparison (Sec. III-E). Every
iteration of Algorithm 1 with alpha M row blocks and gamma N column blocks forms
alpha M gamma N forward and as many back projections of one (row block, column block)
pair, i.e. 2 alpha M gamma N products.

Everything here runs on the device through the library: the least-squares reference is
CGLS on the library's own projectors (FP32 projections, FP64 vector arithmetic) and the
iterates come from `bsgd_step`. Run `python -m paper_1903_11874_amd.study` for the tables.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

from .bsgd import Geometry, Solver


def _zeros(n, device):
    import torch
    return torch.zeros(n, dtype=torch.float32, device=device)


def spectral_norm_sq(geom: Geometry, device, iters: int = 50, seed: int = 0) -> float:
    """Largest eigenvalue of A^T A by power iteration on the library's projectors."""
    import torch
    g = geom.spec
    n = g.nx * g.ny * g.nz
    gen = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.rand(n, generator=gen, dtype=torch.float64).to(device)
    lam = 0.0
    for _ in range(iters):
        v = v / torch.linalg.norm(v)
        w = geom.back_project(geom.forward_project(v.float())).double()
        lam = float(torch.dot(v, w))
        v = w
    return lam


def least_squares(geom: Geometry, y, iters: int = 200, rtol: float = 1e-8):
    """argmin ||y - A x|| by CGLS (conjugate gradients on the normal equations) from x = 0.

    Stops when ||A^T r|| <= rtol ||A^T y|| (r the recurred residual) or after iters steps.
    FP32 projections put a floor near 1e-7 under that ratio, below which the recurrences
    lose conjugacy, so the iterate with the smallest ||A^T r|| is returned (FP64)."""
    import torch
    yd = y.double()
    g = geom.spec
    x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float64, device=y.device)
    r = yd.clone()
    s = geom.back_project(r.float()).double()
    p = s.clone()
    gamma = float(torch.dot(s, s))
    stop = rtol * rtol * gamma
    best, best_gamma = x.clone(), gamma
    for _ in range(iters):
        if gamma <= stop or gamma > 1e4 * best_gamma:
            break
        q = geom.forward_project(p.float()).double()
        alpha = gamma / float(torch.dot(q, q))
        x += alpha * p
        r -= alpha * q
        s = geom.back_project(r.float()).double()
        gamma_new = float(torch.dot(s, s))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        if gamma < best_gamma:
            best, best_gamma = x.clone(), gamma
    return best


def products_per_iteration(rows_per_iter: int, blocks_per_iter: int) -> int:
    """Sub-matrix products per iteration of Algorithm 1: one forward and one back projection
    per selected (row block, column block) pair."""
    return 2 * rows_per_iter * blocks_per_iter


def ds_curve(geom: Geometry, y, x_ref, rows_per_iter: int, blocks_per_iter: int, mu: float,
             n_products: int, n_points: int = 8, seed: int = 1,
             **opts) -> List[Tuple[int, float]]:
    """DS = ||x - x_ref|| at n_points equally spaced iteration counts of one run from x = 0,
    as (products so far, DS) pairs."""
    import torch
    g = geom.spec
    x = _zeros(g.nx * g.ny * g.nz, y.device)
    s = Solver(geom, y, x, rows_per_iter=rows_per_iter, blocks_per_iter=blocks_per_iter,
               mu=mu, seed=seed, **opts)
    per = products_per_iteration(rows_per_iter, blocks_per_iter)
    iters = max(n_products // per, n_points)
    marks = [round(iters * (i + 1) / n_points) for i in range(n_points)]
    out, done = [], 0
    try:
        for m in marks:
            s.step(m - done)
            done = m
            out.append((done * per, float(torch.linalg.norm(x.double() - x_ref.double()))))
    finally:
        s.close()
    return out


def snr_db(x_true, x) -> float:
    import torch
    d = torch.linalg.norm((x_true.double() - x.double()))
    return float(20.0 * torch.log10(torch.linalg.norm(x_true.double()) / d))


def snr_curve(geom: Geometry, y, x_true, rows_per_iter: int, blocks_per_iter: int, mu: float,
              effective_epochs: int, n_points: int = 5, seed: int = 1,
              **opts) -> List[Tuple[int, float]]:
    """Image SNR at n_points equally spaced effective epochs (1/(alpha gamma) iterations each)
    of one run from x = 0, as (effective epochs, SNR dB) pairs."""
    g = geom.spec
    x = _zeros(g.nx * g.ny * g.nz, y.device)
    s = Solver(geom, y, x, rows_per_iter=rows_per_iter, blocks_per_iter=blocks_per_iter,
               mu=mu, seed=seed, **opts)
    out, done = [], 0
    try:
        T = s.epoch_iters
        for i in range(n_points):
            e = round(effective_epochs * (i + 1) / n_points)
            s.step((e - done) * T)
            done = e
            out.append((e, snr_db(x_true, x)))
    finally:
        s.close()
    return out


def tune_step(run, scales: Sequence[float]) -> Tuple[float, list]:
    """The scale whose run ends lowest (run(scale) returns a curve of (abscissa, value)
    pairs; non-finite ends lose), as the paper tunes each method for its fastest rate."""
    best = None
    for c in scales:
        curve = run(c)
        end = curve[-1][1]
        if math.isfinite(end) and (best is None or end < best[1][-1][1]):
            best = (c, curve)
    if best is None:
        raise RuntimeError("every step length diverged")
    return best


# --------------------------------------------------------------------------- the tables

E2_PARTITIONS = ((2, 8, 4), (4, 4, 4), (8, 4, 2))   # (M, bx, by): 2x32, 4x16, 8x8 blocks
GAMMA_PAIRS = ((4, 1), (2, 2), (1, 4))               # (alpha M, gamma N) at four pairs
STEP_SCALES = (0.5, 1.0, 2.0, 4.0)                   # mu = scale / (2 ||A||^2)


def _study_inputs(name: str, device):
    import numpy as np
    import torch
    from bsgd_inputs.configs import STUDY_2D, study_geometry
    from bsgd_inputs.phantoms import add_gaussian_noise_snr, ellipse_phantom_2d
    d = STUDY_2D[name]
    geom = Geometry(study_geometry(name, 1, 1, 1))
    x_true = ellipse_phantom_2d(d["nx"], d["nx"], d["n_shapes"], d["phantom_seed"]).ravel()
    xt = torch.tensor(x_true, dtype=torch.float32, device=device)
    ax = geom.forward_project(xt).double().cpu().numpy()
    y = add_gaussian_noise_snr(ax, d["snr_db"], d["noise_seed"])
    return geom, xt, torch.tensor(np.asarray(y), dtype=torch.float32, device=device)


def partition_study(device, n_products: int = 8000, scales=STEP_SCALES) -> Dict:
    """Sec. III-A and III-B on the 16x16 setup: alpha = gamma = 1 at M = 4, N = 2, then
    64 blocks cut as 2x32, 4x16 and 8x8 with one pair per iteration, each at its best
    step length; DS against products."""
    from bsgd_inputs.configs import study_geometry
    g0, _, y = _study_inputs("e1", device)
    x_lsq = least_squares(g0, y)
    L = spectral_norm_sq(g0, device)
    ds0 = float(x_lsq.norm())
    rows = {}
    geom = Geometry(study_geometry("e1", 4, 2, 1))
    rows["4x2 alpha=gamma=1"] = tune_step(
        lambda c: ds_curve(geom, y, x_lsq, 4, 2, c / (2 * L), n_products), scales)
    for M, bx, by in E2_PARTITIONS:
        geom = Geometry(study_geometry("e1", M, bx, by))
        rows[f"{M}x{bx * by} one pair"] = tune_step(
            lambda c: ds_curve(geom, y, x_lsq, 1, 1, c / (2 * L), n_products), scales)
    return {"ds0": ds0, "L": L, "rows": rows}


def gamma_study(device, n_products: int = 8000, M: int = 4, bx: int = 4, by: int = 4,
                scales=STEP_SCALES) -> Dict:
    """Sec. III-C: four pairs per iteration at fixed M and N, from gamma N = 1 to 4."""
    from bsgd_inputs.configs import study_geometry
    g0, _, y = _study_inputs("e1", device)
    x_lsq = least_squares(g0, y)
    L = spectral_norm_sq(g0, device)
    geom = Geometry(study_geometry("e1", M, bx, by))
    rows = {}
    for R, B in GAMMA_PAIRS:
        rows[f"alpha M={R} gamma N={B}"] = tune_step(
            lambda c: ds_curve(geom, y, x_lsq, R, B, c / (2 * L), n_products), scales)
    return {"ds0": float(x_lsq.norm()), "L": L, "rows": rows}


def tv_study(device, effective_epochs: int = 500, tv_lambda: float = 100.0,
             mu_scale: float = 1.0) -> Dict:
    """Sec. III-E TV comparison on the 64x64 setup: BSGD-TV with M = 20, N = 4,
    alpha = 0.05, gamma = 0.5 against gradient descent (alpha = gamma = 1, no TV) at the
    same step length; image SNR against effective epochs."""
    from bsgd_inputs.configs import study_geometry
    g0, xt, y = _study_inputs("e6", device)
    L = spectral_norm_sq(g0, device)
    mu = mu_scale / (2 * L)
    geom = Geometry(study_geometry("e6", 20, 2, 2, partition_seed=6))
    return {"L": L, "mu": mu, "rows": {
        "BSGD-TV": snr_curve(geom, y, xt, 1, 2, mu, effective_epochs, tv_lambda=tv_lambda),
        "GD": snr_curve(geom, y, xt, 20, 4, mu, effective_epochs),
    }}


def main(argv=None):
    import argparse
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--products", type=int, default=8000)
    ap.add_argument("--epochs", type=int, default=500)
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    for title, res in (("partitions (16x16, 64 blocks)", partition_study(dev, a.products)),
                       ("gamma at M=4, N=16, four pairs", gamma_study(dev, a.products))):
        print(f"{title}: DS0 = {res['ds0']:.4g}")
        for name, (c, curve) in res["rows"].items():
            pts = "  ".join(f"{p}:{v:.3g}" for p, v in curve)
            print(f"  {name:22s} mu = {c:g}/(2L)  {pts}")
    res = tv_study(dev, a.epochs)
    print(f"TV comparison (64x64), mu = {res['mu']:.3g}")
    for name, curve in res["rows"].items():
        print(f"  {name:8s} " + "  ".join(f"{e}:{v:.2f} dB" for e, v in curve))


if __name__ == "__main__":
    main()
