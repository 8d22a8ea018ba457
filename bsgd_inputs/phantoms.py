"""Seeded random-ellipse / ellipsoid phantoms and measurement-noise models.

Phantoms are point-sampled at voxel centres: each shape adds its intensity where
the centre lies inside it, the shapes are summed and the result is clipped at 0.
Coordinates are normalised so that the unit disc (ball) is the circle (sphere)
inscribed in the image. Draw order is fixed (documented per function) so a seed
determines the phantom exactly; the generator is numpy's PCG64.
"""
from __future__ import annotations

import numpy as np

from .configs import GeometrySpec, Workload


def _ellipse_params(rng: np.random.Generator, n: int):
    shapes = []
    for _ in range(n):
        rho = np.sqrt(rng.uniform(0.0, 1.0))      # area-uniform radius in the unit disc
        phi = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        ang = rng.uniform(0.0, np.pi)
        val = rng.uniform(-0.3, 1.0)
        shapes.append((rho * np.cos(phi), rho * np.sin(phi), a, b, ang, val))
    return shapes


def ellipse_phantom_2d(nx: int, ny: int, n_shapes: int, seed: int, return_shapes: bool = False):
    """2D phantom [ny][nx] float64; shapes are (cx, cy, a, b, angle, value) in unit-disc units.

    Per shape the draws are: U(0,1) for the radius (sqrt for area uniformity),
    U(0, 2 pi) for the polar angle, U(0.05,0.4) twice for the semi-axes,
    U(0, pi) for the orientation and U(-0.3, 1.0) for the intensity.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = _ellipse_params(rng, n_shapes)
    half = 0.5 * min(nx, ny)
    xs = (np.arange(nx) - (nx - 1) / 2.0) / half
    ys = (np.arange(ny) - (ny - 1) / 2.0) / half
    X, Y = np.meshgrid(xs, ys)  # [ny][nx]
    img = np.zeros((ny, nx))
    for cx, cy, a, b, ang, val in shapes:
        c, s = np.cos(ang), np.sin(ang)
        px, py = X - cx, Y - cy
        u = (c * px + s * py) / a
        v = (-s * px + c * py) / b
        img[u * u + v * v <= 1.0] += val
    img = np.maximum(img, 0.0)
    return (img, shapes) if return_shapes else img


def _random_rotation(rng: np.random.Generator):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_phantom_3d(nx: int, ny: int, nz: int, n_shapes: int, seed: int,
                         return_shapes: bool = False):
    """3D phantom [nz][ny][nx] float64.

    Per shape the draws are: a centre uniform in the unit ball (radius U^(1/3),
    direction from a normalised 3-vector of standard normals), three semi-axes
    U(0.05, 0.4), a uniformly random rotation (normalised 4-vector of standard
    normals read as a quaternion) and an intensity U(-0.3, 1.0). Shapes are
    (centre[3], axes[3], rotation[3x3], value).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = []
    for _ in range(n_shapes):
        r = rng.uniform(0.0, 1.0) ** (1.0 / 3.0)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        centre = r * d
        axes = rng.uniform(0.05, 0.4, size=3)
        rot = _random_rotation(rng)
        val = rng.uniform(-0.3, 1.0)
        shapes.append((centre, axes, rot, val))
    half = 0.5 * min(nx, ny, nz)
    xs = (np.arange(nx) - (nx - 1) / 2.0) / half
    ys = (np.arange(ny) - (ny - 1) / 2.0) / half
    zs = (np.arange(nz) - (nz - 1) / 2.0) / half
    img = np.zeros((nz, ny, nx))
    Y, X = np.meshgrid(ys, xs, indexing="ij")  # [ny][nx]
    for centre, axes, rot, val in shapes:
        for k in range(nz):
            p = np.stack([X - centre[0], Y - centre[1], np.full_like(X, zs[k] - centre[2])], axis=-1)
            loc = p @ rot  # coordinates in the shape's own frame
            q = (loc[..., 0] / axes[0]) ** 2 + (loc[..., 1] / axes[1]) ** 2 + (loc[..., 2] / axes[2]) ** 2
            img[k][q <= 1.0] += val
    img = np.maximum(img, 0.0)
    return (img, shapes) if return_shapes else img


def phantom_for(g: GeometrySpec, n_shapes: int, seed: int) -> np.ndarray:
    """Phantom shaped like the geometry's image, flattened in [z][y][x] order (float64)."""
    if g.is_3d:
        return ellipsoid_phantom_3d(g.nx, g.ny, g.nz, n_shapes, seed).reshape(-1)
    return ellipse_phantom_2d(g.nx, g.ny, n_shapes, seed).reshape(-1)


def random_image(n: int, seed: int, low: float = 0.0, high: float = 1.0) -> np.ndarray:
    """A seeded uniform random vector (used as generic image / residual inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(low, high, size=n)


def add_gaussian_noise(y: np.ndarray, rel_sigma: float, seed: int) -> np.ndarray:
    """y + N(0, (rel_sigma * max y)^2), one draw per entry in memory order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sigma = rel_sigma * float(np.max(y))
    return y + rng.normal(0.0, sigma, size=y.shape)


def add_gaussian_noise_snr(y: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """y + e with white Gaussian e scaled so that 20 log10(||y|| / ||e||) = snr_db."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.normal(size=y.shape)
    e *= np.linalg.norm(y) / (np.linalg.norm(e) * 10.0 ** (snr_db / 20.0))
    return y + e


def poisson_log_noise(y: np.ndarray, incident: float, seed: int) -> np.ndarray:
    """Transmission noise on line integrals y.

    Line integrals are scaled by kappa = 4 / max(y) to attenuation units, photon
    counts ~ Poisson(incident exp(-kappa y)) clamped to >= 1, then log-transformed
    back: y' = -ln(counts / incident) / kappa.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kappa = 4.0 / float(np.max(y))
    counts = rng.poisson(incident * np.exp(-kappa * y)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    return -np.log(counts / incident) / kappa
