"""Total variation and its proximal step, as used by BSGD-TV (Algorithm 4).

TEST INFRASTRUCTURE (oracle), FP64.

* TV (Sec. II-B, the equation after Eq. (TVequ)): isotropic, backward differences,
  TV(x) = sum over voxels of || (x_c - x_{c-1 along each axis}) ||_2. The paper
  writes the 2D case; the 3D case adds the third difference. Differences across
  the low boundary are taken as zero (Neumann reading).
* Prox (Algorithm 4, denoising step): t = argmin ||t - x||^2 + 2 mu lambda TV(t),
  i.e. argmin 1/2 ||t - x||^2 + w TV(t) with w = mu lambda. The paper names no
  solver (it points to ISTA/FISTA-style TV denoising); the reading used here is
  the fast gradient projection (FGP) method of Beck and Teboulle (IEEE TIP 2009)
  on the dual: p lives in the unit ball per voxel, t = x - w D^T p, and K
  accelerated projected-gradient steps of size 1/(4 dim w) are taken from p = 0.

Pinned by: identity at w = 0, invariance of constant images, the closed-form
prox of a two-level 1D step, an exact box-constrained QP solve of the 1D dual,
and weak duality (primal - dual gap >= 0, shrinking with K).
"""
from __future__ import annotations

import math

import numpy as np


def grad(x: np.ndarray) -> np.ndarray:
    """Backward differences D x: shape (ndim, *x.shape); zero at the low boundary of each axis."""
    out = np.zeros((x.ndim,) + x.shape)
    for a in range(x.ndim):
        sl_hi = [slice(None)] * x.ndim
        sl_lo = [slice(None)] * x.ndim
        sl_hi[a] = slice(1, None)
        sl_lo[a] = slice(0, -1)
        out[a][tuple(sl_hi)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
    return out


def grad_adjoint(p: np.ndarray) -> np.ndarray:
    """D^T p, the adjoint of ``grad``: <D x, p> = <x, D^T p>."""
    nd = p.shape[0]
    out = np.zeros(p.shape[1:])
    for a in range(nd):
        sl_hi = [slice(None)] * nd
        sl_lo = [slice(None)] * nd
        sl_hi[a] = slice(1, None)
        sl_lo[a] = slice(0, -1)
        out[tuple(sl_hi)] += p[a][tuple(sl_hi)]
        out[tuple(sl_lo)] -= p[a][tuple(sl_hi)]
    return out


def tv(x: np.ndarray) -> float:
    return float(np.sum(np.sqrt(np.sum(grad(x) ** 2, axis=0))))


def project_unit_ball(p: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.sum(p * p, axis=0))
    return p / np.maximum(1.0, nrm)[None]


def fgp_prox(b: np.ndarray, w: float, iters: int = 20, return_dual: bool = False):
    """Approximate argmin_t 1/2 ||t - b||^2 + w TV(t) with ``iters`` FGP steps."""
    b = np.asarray(b, dtype=np.float64)
    if w == 0.0 or iters <= 0:
        out = b.copy()
        return (out, np.zeros((b.ndim,) + b.shape)) if return_dual else out
    nd = b.ndim
    step = 1.0 / (4.0 * nd * w)
    p = np.zeros((nd,) + b.shape)
    r = p.copy()
    tk = 1.0
    for _ in range(iters):
        u = b - w * grad_adjoint(r)
        p_new = project_unit_ball(r + step * grad(u))
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * tk * tk)) / 2.0
        r = p_new + ((tk - 1.0) / t_new) * (p_new - p)
        p, tk = p_new, t_new
    out = b - w * grad_adjoint(p)
    return (out, p) if return_dual else out


def primal_objective(t: np.ndarray, b: np.ndarray, w: float) -> float:
    return 0.5 * float(np.sum((t - b) ** 2)) + w * tv(t)


def dual_objective(p: np.ndarray, b: np.ndarray, w: float) -> float:
    """Dual of the prox problem at a feasible p (|p| <= 1 per voxel)."""
    u = b - w * grad_adjoint(p)
    return 0.5 * float(np.sum(b * b)) - 0.5 * float(np.sum(u * u))
