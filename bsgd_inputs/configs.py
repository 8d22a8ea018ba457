"""Workload descriptions: scan geometries, block partitions and solver settings.

Everything here is plain data. Geometry conventions (shared by every consumer):

* The volume is centred at the origin; voxel (i, j, k) has centre
  ((i - (nx-1)/2) vx, (j - (ny-1)/2) vy, (k - (nz-1)/2) vz); image memory is
  [z][y][x] with x fastest.
* View angle theta_m = m * span / n_views.
* Fan and cone beam: the source sits at sod (cos t, sin t, 0); the flat detector is
  centred at -(sdd - sod) (cos t, sin t, 0) with u-axis (-sin t, cos t, 0) and
  v-axis (0, 0, 1); detector pixel (k, l) is centred at u = (k - (nu-1)/2) du,
  v = (l - (nv-1)/2) dv.
* Parallel beam (2D): ray k passes through u_k (-sin t, cos t) with direction
  (cos t, sin t).
* Sinogram memory is [view][v][u] with u fastest; 2D geometries have nz = nv = 1.
* Column blocks are a regular bx x by x bz tiling of the voxel grid (tile t of an
  axis with n voxels and b tiles covers [floor(t n / b), floor((t+1) n / b))), with
  block index j = (tz by + ty) bx + tx.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, Optional, Tuple

KINDS = ("parallel2d", "fan2d", "cone3d")
IM_MODES = ("none", "colnorm", "area", "uniform")


@dataclass(frozen=True)
class GeometrySpec:
    kind: str
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    n_views: int
    angle_span: float  # radians
    nu: int
    nv: int
    du: float
    dv: float
    sod: float = 0.0
    sdd: float = 0.0
    bx: int = 1
    by: int = 1
    bz: int = 1
    n_row_blocks: int = 1
    partition_seed: int = 0
    su: int = 1
    sv: int = 1
    im_mode: str = "none"

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"unknown geometry kind {self.kind!r}")
        if self.im_mode not in IM_MODES:
            raise ValueError(f"unknown importance-sampling mode {self.im_mode!r}")

    @property
    def is_3d(self) -> bool:
        return self.kind == "cone3d"

    @property
    def n_blocks(self) -> int:
        return self.bx * self.by * self.bz

    @property
    def n_subdet(self) -> int:
        return self.su * self.sv

    def angles(self):
        import numpy as np
        return np.arange(self.n_views, dtype=np.float64) * (self.angle_span / self.n_views)

    def with_(self, **kw) -> "GeometrySpec":
        return replace(self, **kw)


@dataclass(frozen=True)
class SolverSpec:
    rows_per_iter: int = 1      # alpha * M
    blocks_per_iter: int = 1    # gamma * N
    effective_epochs: int = 1
    seed: int = 12345
    mu_scale: float = 0.5       # mu = mu_scale / (2 L), L = sigma_max(A)^2
    tv_lambda: float = 0.0
    tv_inner_iters: int = 20


@dataclass(frozen=True)
class Workload:
    name: str
    geometry: GeometrySpec
    solver: SolverSpec
    phantom_seed: int
    n_shapes: int
    noise: str            # "gaussian" | "poisson" | "none"
    noise_level: float    # relative sigma for gaussian, incident photons for poisson
    noise_seed: int
    description: str = ""


def ray_count(g: GeometrySpec) -> int:
    return g.n_views * g.nv * g.nu


def voxel_count(g: GeometrySpec) -> int:
    return g.nx * g.ny * g.nz


_C1 = Workload(
    name="c1_parallel64",
    geometry=GeometrySpec(kind="parallel2d", nx=64, ny=64, nz=1, vx=1.0, vy=1.0, vz=1.0,
                          n_views=90, angle_span=math.pi, nu=96, nv=1, du=1.0, dv=1.0,
                          bx=4, by=4, bz=1, n_row_blocks=9, partition_seed=11),
    solver=SolverSpec(rows_per_iter=1, blocks_per_iter=1, effective_epochs=20, seed=101),
    phantom_seed=1001, n_shapes=10, noise="gaussian", noise_level=0.01, noise_seed=2001,
    description="2D parallel beam 64x64 @1 mm, 90 views over [0,180) deg, 96 bins @1 mm, "
                "4x4 image blocks, 9 angle subsets, 20 epochs",
)

_C2 = Workload(
    name="c2_fan512_im",
    geometry=GeometrySpec(kind="fan2d", nx=512, ny=512, nz=1, vx=0.5, vy=0.5, vz=0.5,
                          n_views=720, angle_span=2 * math.pi, nu=768, nv=1, du=1.0, dv=1.0,
                          sod=500.0, sdd=1000.0, bx=8, by=8, bz=1, n_row_blocks=16,
                          partition_seed=12, su=4, sv=1, im_mode="colnorm"),
    solver=SolverSpec(rows_per_iter=1, blocks_per_iter=64, effective_epochs=50, seed=102),
    phantom_seed=1002, n_shapes=24, noise="poisson", noise_level=1e5, noise_seed=2002,
    description="2D fan beam 512x512 @0.5 mm, 720 views over 360 deg, 768 bins @1 mm, "
                "SOD 500, SDD 1000, 8x8 image blocks, 16 angle subsets, importance sampling "
                "by block column norms over 4 sub-detectors, 50 epochs",
)

_C3 = Workload(
    name="c3_cone256_tv",
    geometry=GeometrySpec(kind="cone3d", nx=256, ny=256, nz=256, vx=0.5, vy=0.5, vz=0.5,
                          n_views=360, angle_span=2 * math.pi, nu=384, nv=384, du=1.0, dv=1.0,
                          sod=600.0, sdd=1200.0, bx=4, by=4, bz=16, n_row_blocks=24,
                          partition_seed=13, su=2, sv=2, im_mode="none"),
    solver=SolverSpec(rows_per_iter=1, blocks_per_iter=64, effective_epochs=30, seed=103,
                      tv_lambda=1e-3, tv_inner_iters=20),
    phantom_seed=1003, n_shapes=32, noise="gaussian", noise_level=0.01, noise_seed=2003,
    description="3D cone beam 256^3 @0.5 mm, 360 views over 360 deg, 384x384 detector @1 mm, "
                "SOD 600, SDD 1200, 16 axial slabs x 4x4 tiles, 24 angle subsets, TV 1e-3, 30 epochs",
)

_C5 = Workload(
    name="c5_cone128",
    geometry=GeometrySpec(kind="cone3d", nx=128, ny=128, nz=128, vx=1.0, vy=1.0, vz=1.0,
                          n_views=180, angle_span=2 * math.pi, nu=192, nv=192, du=2.0, dv=2.0,
                          sod=600.0, sdd=1200.0, bx=2, by=2, bz=2, n_row_blocks=6,
                          partition_seed=15),
    solver=SolverSpec(rows_per_iter=6, blocks_per_iter=8, effective_epochs=1, seed=105,
                      tv_lambda=1e-3),
    phantom_seed=1005, n_shapes=32, noise="gaussian", noise_level=0.01, noise_seed=2005,
    description="3D cone beam 128^3 @1 mm, 180 views of a 192x192 detector @2 mm",
)


def fan_request_geometry(side: int) -> GeometrySpec:
    """Serving-mix request geometry: fan beam, views = bins = 1.5 side over 360 deg."""
    n = int(round(1.5 * side))
    return GeometrySpec(kind="fan2d", nx=side, ny=side, nz=1, vx=256.0 / side, vy=256.0 / side,
                        vz=256.0 / side, n_views=n, angle_span=2 * math.pi, nu=n, nv=1,
                        du=768.0 / n, dv=1.0, sod=500.0, sdd=1000.0, bx=8, by=8, bz=1,
                        n_row_blocks=16, partition_seed=14)


WORKLOADS: Dict[str, Workload] = {w.name: w for w in (_C1, _C2, _C3, _C5)}
SERVING_SIDES = (128, 256, 384, 512, 768, 1024)


def workload(name: str) -> Workload:
    return WORKLOADS[name]


# The paper's 2D convergence-study setups (Sec. III-A to III-D and the TV comparison of
# Sec. III-E), with image and detector pixels of size 1 as the paper states for its 2D work.
STUDY_2D = {
    # 16x16 image, source and detector both 50 from the centre, 30 bins, 10 degree steps
    # over a full turn: A is 1080 x 256. Data SNR 17.5 dB.
    "e1": dict(nx=16, n_views=36, angle_span=2 * math.pi, nu=30, sod=50.0, sdd=100.0,
               n_shapes=6, phantom_seed=5, snr_db=17.5, noise_seed=8),
    # 64x64 image, source and detector both 100 from the centre, 180 bins, 1 degree steps
    # over half a turn: A is 32400 x 4096. Data SNR 28.8 dB.
    "e6": dict(nx=64, n_views=180, angle_span=math.pi, nu=180, sod=100.0, sdd=200.0,
               n_shapes=10, phantom_seed=21, snr_db=28.8, noise_seed=8),
}


def study_geometry(name: str, n_row_blocks: int, bx: int, by: int,
                   partition_seed: int = 3) -> GeometrySpec:
    """Fan-beam geometry of a 2D study setup cut into n_row_blocks x (bx by) blocks."""
    d = STUDY_2D[name]
    return GeometrySpec(kind="fan2d", nx=d["nx"], ny=d["nx"], nz=1, vx=1.0, vy=1.0, vz=1.0,
                        n_views=d["n_views"], angle_span=d["angle_span"], nu=d["nu"], nv=1,
                        du=1.0, dv=1.0, sod=d["sod"], sdd=d["sdd"], bx=bx, by=by, bz=1,
                        n_row_blocks=n_row_blocks, partition_seed=partition_seed)
