"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds workload descriptions (plain numbers) and seeded generators
of phantoms and measurement noise. It contains none of the reconstruction
method's arithmetic: no projection, no back projection, no solver step.
"""
from .configs import (GeometrySpec, SolverSpec, Workload, WORKLOADS, workload, ray_count, voxel_count,
                      STUDY_2D, study_geometry)
from .phantoms import (ellipse_phantom_2d, ellipsoid_phantom_3d, phantom_for, add_gaussian_noise,
                       add_gaussian_noise_snr, poisson_log_noise, random_image)

__all__ = [
    "GeometrySpec", "SolverSpec", "Workload", "WORKLOADS", "workload", "ray_count", "voxel_count",
    "ellipse_phantom_2d", "ellipsoid_phantom_3d", "phantom_for", "add_gaussian_noise",
    "poisson_log_noise", "random_image", "STUDY_2D", "study_geometry", "add_gaussian_noise_snr",
]
