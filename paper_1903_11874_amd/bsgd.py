"""Python binding of the BSGD C ABI (include/bsgd.h).

Argument marshalling only: every step of the method runs in the HIP library
libbsgd.so. PyTorch supplies device memory and the current stream. The binding
refuses to work when the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsgd.so")

BSGD_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_UNSUPPORTED", 3: "E_OUT_OF_MEMORY", 4: "E_DEVICE",
                5: "E_DIVERGED", 6: "E_STATE"}
KIND = {"parallel2d": 0, "fan2d": 1, "cone3d": 2}
IM_MODE = {"none": 0, "colnorm": 1, "area": 2, "uniform": 3}
TABLE = {"view_order": 0, "group_start": 1, "im_weights": 2, "im_table": 3, "nnz": 4, "footprint": 5,
         "im_area": 6}
KERNELS = ("forward_project", "residual", "back_project_step", "tv_prox", "draws")
ACCUMULATE = 1


class BsgdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bsgd {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("n_views", ctypes.c_int32), ("angles_rad", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32), ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
        ("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32),
        ("n_row_blocks", ctypes.c_int32), ("partition_seed", ctypes.c_uint64),
        ("su", ctypes.c_int32), ("sv", ctypes.c_int32), ("im_mode", ctypes.c_int32),
        ("im_table", ctypes.POINTER(ctypes.c_uint32)),
        ("allocator", ctypes.POINTER(Allocator)),
    ]


class GeometryInfo(ctypes.Structure):
    _fields_ = [
        ("n_rays", ctypes.c_int64), ("n_voxels", ctypes.c_int64), ("n_blocks", ctypes.c_int32),
        ("n_row_blocks", ctypes.c_int32), ("n_subdet", ctypes.c_int32), ("max_group_views", ctypes.c_int32),
        ("z_floats", ctypes.c_int64), ("nnz", ctypes.c_int64),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("rows_per_iter", ctypes.c_int32), ("blocks_per_iter", ctypes.c_int32), ("node_count", ctypes.c_int32),
        ("tv_inner_iters", ctypes.c_int32), ("mu", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("tv_lambda", ctypes.c_double), ("tv_every", ctypes.c_int32), ("max_effective_epochs", ctypes.c_int32),
        ("tol", ctypes.c_double), ("check_every", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("auto_mu", ctypes.c_int32), ("im_until", ctypes.c_int32), ("mu_eps", ctypes.c_double),
        ("mu_delta", ctypes.c_double), ("mu_t1", ctypes.c_double), ("mu_t2", ctypes.c_double),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("fp_views_per_group", ctypes.c_int32), ("fp_ray_split", ctypes.c_int32),
                ("fp_waves_per_pair", ctypes.c_int32), ("fp_staged", ctypes.c_int32),
                ("bp_waves", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


EXPORTED = (
    "bsgd_geometry_create", "bsgd_geometry_destroy", "bsgd_geometry_get_info", "bsgd_geometry_table",
    "bsgd_forward_project", "bsgd_back_project", "bsgd_solver_create", "bsgd_step", "bsgd_solver_counts",
    "bsgd_solver_last_schedule", "bsgd_solver_state", "bsgd_solver_set_profiling", "bsgd_solver_kernel_times",
    "bsgd_solver_destroy", "bsgd_solve", "bsgd_last_error", "bsgd_step_batch", "bsgd_geometry_set_tuning",
    "bsgd_geometry_get_tuning", "bsgd_solver_step_length", "bsgd_normal_residual",
    "bsgd_normal_residual_noalloc", "bsgd_noalloc_scratch_bytes", "bsgd_normal_residual_async",
)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbsgd.so (raises if it has not been built) and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1903_11874_amd.build`")
    L = ctypes.CDLL(path)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "bsgd_geometry_create": (i32, [ctypes.POINTER(GeometryDesc), P, ctypes.POINTER(P)]),
        "bsgd_geometry_destroy": (None, [P]),
        "bsgd_geometry_get_info": (i32, [P, ctypes.POINTER(GeometryInfo)]),
        "bsgd_geometry_table": (i32, [P, i32, P, ctypes.c_size_t]),
        "bsgd_forward_project": (i32, [P, P, P, P, i32, i32, u32, P]),
        "bsgd_back_project": (i32, [P, P, P, P, i32, i32, ctypes.c_float, u32, P]),
        "bsgd_solver_create": (i32, [P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(P)]),
        "bsgd_step": (i32, [P, i32, ctypes.POINTER(ctypes.c_double)]),
        "bsgd_solver_counts": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32)]),
        "bsgd_solver_last_schedule": (i32, [P, ctypes.POINTER(i32), P, P, P, ctypes.c_size_t]),
        "bsgd_solver_state": (i32, [P, i32, P, ctypes.c_size_t]),
        "bsgd_solver_set_profiling": (i32, [P, i32]),
        "bsgd_solver_kernel_times": (i32, [P, P, P]),
        "bsgd_solver_destroy": (None, [P]),
        "bsgd_solve": (i32, [P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(i32),
                             ctypes.POINTER(ctypes.c_double)]),
        "bsgd_last_error": (ctypes.c_char_p, []),
        "bsgd_step_batch": (i32, [ctypes.POINTER(P), i32, i32, P]),
        "bsgd_geometry_set_tuning": (i32, [P, ctypes.POINTER(Tuning)]),
        "bsgd_geometry_get_tuning": (i32, [P, ctypes.POINTER(Tuning)]),
        "bsgd_solver_step_length": (i32, [P, ctypes.POINTER(ctypes.c_double), P, i32, ctypes.POINTER(i32)]),
        "bsgd_normal_residual": (i32, [ctypes.POINTER(P), i32, i32, P, P]),
        "bsgd_normal_residual_noalloc": (i32, [P, P, P, ctypes.POINTER(ctypes.c_double), P]),
        "bsgd_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "bsgd_normal_residual_async": (i32, [ctypes.POINTER(P), i32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != BSGD_OK:
        msg = load_library().bsgd_last_error()
        raise BsgdError(status, msg.decode() if msg else "")


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _dev_ptr(t, dtype_name="float32"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _views_arg(views):
    if views is None:
        return None, 0, None
    arr = np.ascontiguousarray(np.asarray(views, dtype=np.int32).reshape(-1))
    # an empty list must stay a (non-NULL) list: NULL would select every view
    keep = arr if arr.size else np.zeros(1, dtype=np.int32)
    return keep.ctypes.data_as(ctypes.c_void_p), int(arr.size), keep


def torch_allocator() -> Allocator:
    """bsgd_allocator over PyTorch's caching allocator (device memory of the current
    device, stream-ordered on the stream the library names). The returned structure
    holds the callbacks; keep it alive as long as the geometry and its solvers."""

    def _alloc(ctx, nbytes, stream):
        try:
            import torch
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # the library reports a failed allocation as out of memory
            return None

    def _free(ctx, ptr, stream):
        try:
            import torch
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    return Allocator(None, ALLOC_FN(_alloc), FREE_FN(_free))


class Geometry:
    """A scan geometry, its block partition and sampling tables (bsgd_geometry).
    allocator: None (hipMalloc) or "torch" (PyTorch's caching allocator), used for the
    geometry's tables and the state of every solver created from it."""

    def __init__(self, spec, im_table: Optional[np.ndarray] = None, stream=None, allocator=None):
        self.spec = spec
        lib = load_library()
        angles = np.ascontiguousarray(spec.angles(), dtype=np.float64)
        self._angles = angles
        d = GeometryDesc()
        d.kind = KIND[spec.kind]
        d.nx, d.ny, d.nz = spec.nx, spec.ny, spec.nz
        d.vx, d.vy, d.vz = spec.vx, spec.vy, spec.vz
        d.n_views = spec.n_views
        d.angles_rad = angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.nu, d.nv, d.du, d.dv = spec.nu, spec.nv, spec.du, spec.dv
        d.sod, d.sdd = spec.sod, spec.sdd
        d.bx, d.by, d.bz = spec.bx, spec.by, spec.bz
        d.n_row_blocks = spec.n_row_blocks
        d.partition_seed = spec.partition_seed
        d.su, d.sv = spec.su, spec.sv
        d.im_mode = IM_MODE[spec.im_mode]
        self._im = None
        self._alloc = None
        if allocator == "torch":
            self._alloc = torch_allocator()
            d.allocator = ctypes.pointer(self._alloc)
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        if im_table is not None:
            self._im = np.ascontiguousarray(im_table, dtype=np.uint32)
            d.im_table = self._im.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        h = ctypes.c_void_p()
        _check(lib.bsgd_geometry_create(ctypes.byref(d), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        info = GeometryInfo()
        _check(lib.bsgd_geometry_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in GeometryInfo._fields_}

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load_library().bsgd_geometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _get_tuning(self) -> Tuning:
        t = Tuning()
        _check(load_library().bsgd_geometry_get_tuning(self._h, ctypes.byref(t)))
        return t

    def set_tuning(self, fp_views_per_group: Optional[int] = None, fp_ray_split: Optional[int] = None,
                   fp_waves_per_pair: Optional[int] = None, bp_waves: Optional[int] = None):
        """Launch shapes of the projectors (bsgd_geometry_set_tuning)."""
        t = self._get_tuning()
        if fp_views_per_group is not None:
            t.fp_views_per_group = int(fp_views_per_group)
        if fp_ray_split is not None:
            t.fp_ray_split = int(fp_ray_split)
        if fp_waves_per_pair is not None:
            t.fp_waves_per_pair = int(fp_waves_per_pair)
        if bp_waves is not None:
            t.bp_waves = int(bp_waves)
        _check(load_library().bsgd_geometry_set_tuning(self._h, ctypes.byref(t)))

    @property
    def bp_waves(self) -> int:
        """Waves of a 2D back-projection workgroup (views split over them)."""
        return self._get_tuning().bp_waves

    @property
    def fp_waves_per_pair(self) -> int:
        return self._get_tuning().fp_waves_per_pair

    @property
    def fp_staged(self) -> bool:
        """True when the forward projector stages blocks in LDS."""
        return bool(self._get_tuning().fp_staged)

    @property
    def fp_views_per_group(self) -> int:
        return self._get_tuning().fp_views_per_group

    @fp_views_per_group.setter
    def fp_views_per_group(self, value: int):
        self.set_tuning(fp_views_per_group=value)

    @property
    def fp_ray_split(self) -> int:
        return self._get_tuning().fp_ray_split

    @fp_ray_split.setter
    def fp_ray_split(self, value: int):
        self.set_tuning(fp_ray_split=value)

    def table(self, name: str) -> np.ndarray:
        g = self.spec
        V, S, N, M = g.n_views, g.su * g.sv, g.n_blocks, g.n_row_blocks
        shapes = {"view_order": ((V,), np.int32), "group_start": ((M + 1,), np.int32),
                  "im_weights": ((V, S, N), np.float64), "im_table": ((V, S, N), np.uint32),
                  "im_area": ((V, S, N), np.float64),
                  "nnz": ((V, S, N), np.int64), "footprint": ((V, N, 4), np.int32)}
        shape, dt = shapes[name]
        out = np.zeros(shape, dtype=dt)
        _check(load_library().bsgd_geometry_table(self._h, TABLE[name], out.ctypes.data_as(ctypes.c_void_p),
                                                  out.nbytes))
        return out

    def groups(self):
        order, start = self.table("view_order"), self.table("group_start")
        return [list(order[start[i]:start[i + 1]]) for i in range(len(start) - 1)]

    def forward_project(self, x, views: Optional[Sequence[int]] = None, block: int = -1, out=None,
                        accumulate: bool = False, stream=None):
        import torch
        g = self.spec
        n_sel = g.n_views if views is None else len(views)
        if x.numel() != g.nx * g.ny * g.nz:
            raise ValueError("x has the wrong size")
        if out is None:
            out = torch.zeros(n_sel * g.nv * g.nu, device=x.device, dtype=torch.float32)
        elif out.numel() != n_sel * g.nv * g.nu:
            raise ValueError("out has the wrong size")
        vp, nv, keep = _views_arg(views)
        _check(load_library().bsgd_forward_project(self._h, _dev_ptr(x), _dev_ptr(out), vp,
                                                   nv if views is not None else n_sel, block,
                                                   ACCUMULATE if accumulate else 0, _stream_ptr(stream)))
        return out

    def back_project(self, y, views: Optional[Sequence[int]] = None, block: int = -1, scale: float = 1.0,
                     out=None, accumulate: bool = False, stream=None):
        import torch
        g = self.spec
        n_sel = g.n_views if views is None else len(views)
        if y.numel() != n_sel * g.nv * g.nu:
            raise ValueError("y has the wrong size")
        if out is None:
            out = torch.zeros(g.nx * g.ny * g.nz, device=y.device, dtype=torch.float32)
        elif out.numel() != g.nx * g.ny * g.nz:
            raise ValueError("out has the wrong size")
        vp, nv, keep = _views_arg(views)
        _check(load_library().bsgd_back_project(self._h, _dev_ptr(y), _dev_ptr(out), vp,
                                                nv if views is not None else n_sel, block, float(scale),
                                                ACCUMULATE if accumulate else 0, _stream_ptr(stream)))
        return out


FLAG_EAGER = 1
FLAG_SUBDET_MEMORY = 2


def make_options(rows_per_iter=0, blocks_per_iter=0, node_count=0, mu=0.0, seed=0, tv_lambda=0.0,
                 tv_inner_iters=20, tv_every=0, max_effective_epochs=0, tol=0.0, check_every=0,
                 eager=False, auto_mu=False, mu_eps=0.0, mu_delta=0.0, mu_t1=0.0, mu_t2=0.0,
                 im_until=0, subdet_memory=False) -> Options:
    o = Options()
    o.rows_per_iter, o.blocks_per_iter, o.node_count = rows_per_iter, blocks_per_iter, node_count
    o.tv_inner_iters, o.mu, o.seed, o.tv_lambda, o.tv_every = tv_inner_iters, mu, seed, tv_lambda, tv_every
    o.max_effective_epochs, o.tol, o.check_every = max_effective_epochs, tol, check_every
    o.flags = (FLAG_EAGER if eager else 0) | (FLAG_SUBDET_MEMORY if subdet_memory else 0)
    o.auto_mu, o.im_until = (1 if auto_mu else 0), int(im_until)
    o.mu_eps, o.mu_delta, o.mu_t1, o.mu_t2 = mu_eps, mu_delta, mu_t1, mu_t2
    return o


class Solver:
    """BSGD state for one reconstruction (bsgd_solver); x is updated in place."""

    def __init__(self, geom: Geometry, y, x, stream=None, **opts):
        self.geom = geom
        self.y, self.x = y, x
        self._stream = stream
        self.options = make_options(**opts)
        h = ctypes.c_void_p()
        _check(load_library().bsgd_solver_create(geom.handle, _dev_ptr(y), _dev_ptr(x), ctypes.byref(self.options),
                                                 _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        k, r, b, t = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().bsgd_solver_counts(h, ctypes.byref(k), ctypes.byref(r), ctypes.byref(b),
                                                 ctypes.byref(t)))
        self.rows_per_iter, self.blocks_per_iter, self.epoch_iters = r.value, b.value, t.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().bsgd_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def iterations(self) -> int:
        k = ctypes.c_int64()
        _check(load_library().bsgd_solver_counts(self._h, ctypes.byref(k), None, None, None))
        return k.value

    def step(self, n_iters: int = 1, residual: bool = False):
        out = ctypes.c_double() if residual else None
        _check(load_library().bsgd_step(self._h, int(n_iters), ctypes.byref(out) if residual else None))
        return out.value if residual else None

    def step_length(self):
        """(current mu, list of mu after each Algorithm 3 check)."""
        lib = load_library()
        mu, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib.bsgd_solver_step_length(self._h, ctypes.byref(mu), None, 0, ctypes.byref(n)))
        hist = np.zeros(max(n.value, 1))
        _check(lib.bsgd_solver_step_length(self._h, None, hist.ctypes.data_as(ctypes.c_void_p), n.value, None))
        return mu.value, list(hist[: n.value])

    def last_schedule(self):
        lib = load_library()
        n = ctypes.c_int32()
        _check(lib.bsgd_solver_last_schedule(self._h, ctypes.byref(n), None, None, None, 0))
        n = n.value
        maxv = self.rows_per_iter * self.geom.info["max_group_views"]
        rows = np.zeros((n, self.rows_per_iter), dtype=np.int32)
        blocks = np.zeros((n, self.blocks_per_iter), dtype=np.int32)
        draws = np.zeros((n, maxv, self.blocks_per_iter), dtype=np.int16)
        _check(lib.bsgd_solver_last_schedule(self._h, None, rows.ctypes.data_as(ctypes.c_void_p),
                                             blocks.ctypes.data_as(ctypes.c_void_p),
                                             draws.ctypes.data_as(ctypes.c_void_p), draws.nbytes))
        return rows, blocks, draws

    def state(self, which: str):
        import torch
        idx = {"g": 0, "ghat": 1, "z": 2, "rho": 3}[which]
        g = self.geom.spec
        n = {0: g.nx * g.ny * g.nz, 1: g.n_row_blocks * g.nx * g.ny * g.nz, 2: self.geom.info["z_floats"],
             3: self.geom.info["z_floats"]}[idx]
        out = torch.empty(max(n, 1), device=self.x.device, dtype=torch.float32)
        _check(load_library().bsgd_solver_state(self._h, idx, _dev_ptr(out), out.numel() * 4))
        return out[:n]

    def set_profiling(self, on: bool = True):
        _check(load_library().bsgd_solver_set_profiling(self._h, 1 if on else 0))

    def kernel_times(self):
        ms = np.zeros(5, dtype=np.float64)
        n = np.zeros(5, dtype=np.int64)
        _check(load_library().bsgd_solver_kernel_times(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                                       n.ctypes.data_as(ctypes.c_void_p)))
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(KERNELS)}


def step_batch(solvers, n_iters: int, stream=None):
    """n_iters iterations of every solver with shared launches (bsgd_step_batch)."""
    arr = (ctypes.c_void_p * len(solvers))(*[s._h.value for s in solvers])
    _check(load_library().bsgd_step_batch(arr, len(solvers), int(n_iters), _stream_ptr(stream)))


def normal_residual(solvers, relative: bool = True, stream=None):
    """||A^T (y - A x)|| (divided by ||A^T y|| when relative) of each solver's current
    image, with one synchronisation (bsgd_normal_residual)."""
    arr = (ctypes.c_void_p * len(solvers))(*[s._h.value for s in solvers])
    out = np.zeros(len(solvers), dtype=np.float64)
    _check(load_library().bsgd_normal_residual(arr, len(solvers), int(bool(relative)),
                                               out.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
    return out


def normal_residual_async(solvers, out_sq, stream=None):
    """Enqueue ||A^T (y - A x)||^2 and ||A^T y||^2 of each solver into out_sq (a page-locked
    float64 host tensor of 2 n values), without waiting (bsgd_normal_residual_async);
    read out_sq after the stream has passed this point."""
    import torch
    if not (isinstance(out_sq, torch.Tensor) and out_sq.dtype == torch.float64 and not out_sq.is_cuda
            and out_sq.is_contiguous() and out_sq.numel() >= 2 * len(solvers)):
        raise ValueError("out_sq must be a contiguous float64 host tensor of at least 2 n values")
    arr = (ctypes.c_void_p * len(solvers))(*[s._h.value for s in solvers])
    _check(load_library().bsgd_normal_residual_async(arr, len(solvers), ctypes.c_void_p(out_sq.data_ptr()),
                                                     _stream_ptr(stream)))


def normal_residual_noalloc(geom: Geometry, y, x, stream=None) -> float:
    """||A^T (y - A x)|| through the allocation-free entry point
    (bsgd_normal_residual_noalloc: static device scratch, no allocation)."""
    out = ctypes.c_double()
    _check(load_library().bsgd_normal_residual_noalloc(geom.handle, _dev_ptr(y), _dev_ptr(x), ctypes.byref(out),
                                                       _stream_ptr(stream)))
    return out.value


def noalloc_scratch_bytes() -> int:
    return int(load_library().bsgd_noalloc_scratch_bytes())


def solve(geom: Geometry, y, x, stream=None, **opts):
    """Run the solver to its stopping rule (bsgd_solve); returns (iterations, ||r||)."""
    o = make_options(**opts)
    it, rn = ctypes.c_int32(), ctypes.c_double()
    _check(load_library().bsgd_solve(geom.handle, _dev_ptr(y), _dev_ptr(x), ctypes.byref(o), _stream_ptr(stream),
                                     ctypes.byref(it), ctypes.byref(rn)))
    return it.value, rn.value
