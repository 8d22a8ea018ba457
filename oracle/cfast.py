"""ctypes front end of the plain C FP64 Siddon projector (oracle/csiddon.c).

TEST INFRASTRUCTURE (oracle). ``build()`` compiles the C file with gcc; the
loaders build it only when no library exists yet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from bsgd_inputs.configs import GeometrySpec
from .geometry import grid_of, ray_endpoints

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csiddon.c")
_LIB = os.path.join(_HERE, "liboracle_siddon.so")
_lib = None


def build() -> str:
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_fp.restype = i64
        L.oracle_fp.argtypes = [ctypes.c_int, P, P, P, i64, P, P, P, P, ctypes.c_int]
        L.oracle_bp.restype = None
        L.oracle_bp.argtypes = [ctypes.c_int, P, P, P, i64, P, P, P, P, ctypes.c_int]
        L.oracle_ray.restype = i64
        L.oracle_ray.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, i64]
        L.oracle_count.restype = None
        L.oracle_count.argtypes = [ctypes.c_int, P, P, P, i64, P, P, P, ctypes.c_int]
        L.oracle_fill.restype = None
        L.oracle_fill.argtypes = [ctypes.c_int, P, P, P, i64, P, P, P, P, P, ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Projector:
    """Matrix-free FP64 A and A^T for one geometry (optionally a subset of rays)."""

    def __init__(self, g: GeometrySpec, rays=None):
        self.g = g
        grid = grid_of(g)
        self.dim = grid.dim
        self.n = np.array(grid.n, dtype=np.int64)
        self.lo = np.array(grid.lo, dtype=np.float64)
        self.v = np.array(grid.v, dtype=np.float64)
        p0, p1 = ray_endpoints(g, rays)
        self.p0 = np.ascontiguousarray(p0)
        self.p1 = np.ascontiguousarray(p1)
        self.n_rays = self.p0.shape[0]
        self.n_vox = int(np.prod(self.n))

    def _args(self):
        return (self.dim, _ptr(self.n), _ptr(self.lo), _ptr(self.v), self.n_rays,
                _ptr(self.p0), _ptr(self.p1))

    def fp(self, x, threads: int = 0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.n_vox
        y = np.zeros(self.n_rays)
        nnz = lib().oracle_fp(*self._args(), _ptr(x), _ptr(y), threads)
        self.last_nnz = int(nnz)
        return y

    def bp(self, r, threads: int = 0):
        r = np.ascontiguousarray(r, dtype=np.float64)
        assert r.size == self.n_rays
        out = np.zeros(self.n_vox)
        lib().oracle_bp(*self._args(), _ptr(r), _ptr(out), threads)
        return out

    def counts(self, threads: int = 0):
        c = np.zeros(self.n_rays, dtype=np.int64)
        lib().oracle_count(*self._args(), _ptr(c), threads)
        return c

    def matrix(self, threads: int = 0) -> sp.csr_matrix:
        counts = self.counts(threads)
        indptr = np.zeros(self.n_rays + 1, dtype=np.int64)
        np.cumsum(counts, out=indptr[1:])
        nnz = int(indptr[-1])
        indices = np.zeros(nnz, dtype=np.int64)
        data = np.zeros(nnz)
        lib().oracle_fill(*self._args(), _ptr(indptr), _ptr(indices), _ptr(data), threads)
        A = sp.csr_matrix((data, indices, indptr), shape=(self.n_rays, self.n_vox))
        A.sum_duplicates()
        return A


def max_threads() -> int:
    return int(lib().oracle_max_threads())
