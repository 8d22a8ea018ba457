"""Explicit sparse system matrix A for small grids.

TEST INFRASTRUCTURE (oracle), FP64. Row i is ray i ([view][v][u] order), column j
is voxel j ([z][y][x] order), entries are the Siddon intersection lengths
(Sec. I after Eq. (yax)). ``matrix_python`` uses the pure-Python Siddon;
``matrix`` uses the C restatement (same definition, faster); the tests check
that the two agree.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from bsgd_inputs.configs import GeometrySpec
from .geometry import grid_of, ray_endpoints
from .siddon import siddon_ray


def matrix_python(g: GeometrySpec) -> sp.csr_matrix:
    grid = grid_of(g)
    p0, p1 = ray_endpoints(g)
    rows, cols, vals = [], [], []
    for i in range(p0.shape[0]):
        idx, ln = siddon_ray(p0[i], p1[i], grid)
        rows.append(np.full(idx.shape, i, dtype=np.int64))
        cols.append(idx)
        vals.append(ln)
    n_vox = int(np.prod(grid.n))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(p0.shape[0], n_vox))
    A.sum_duplicates()
    return A


def matrix(g: GeometrySpec) -> sp.csr_matrix:
    from .cfast import Projector
    return Projector(g).matrix()
