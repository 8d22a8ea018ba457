"""The C-ABI library loads, exports every declared entry point, and rejects bad
arguments before touching the device (no GPU needed for any of this)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsgd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsgd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1903_11874_amd.bsgd import load_library, LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1903_11874_amd.build import build
        build()
    return load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_1903_11874_amd.bsgd import EXPORTED
    assert sorted(EXPORTED) == names


def test_struct_layouts_match_header():
    import subprocess
    import tempfile
    from paper_1903_11874_amd.bsgd import Allocator, GeometryDesc, Options, GeometryInfo, Tuning
    src = '#include "%s"\n#include <stdio.h>\n#include <stddef.h>\nint main(){printf("%%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu", ' \
          'sizeof(bsgd_geometry_desc), sizeof(bsgd_options), sizeof(bsgd_geometry_info), ' \
          'offsetof(bsgd_geometry_desc, im_table), offsetof(bsgd_options, tol), sizeof(bsgd_tuning), ' \
          'offsetof(bsgd_tuning, fp_ray_split), offsetof(bsgd_geometry_desc, allocator), sizeof(bsgd_allocator), ' \
          'offsetof(bsgd_tuning, fp_waves_per_pair), offsetof(bsgd_tuning, fp_staged), offsetof(bsgd_tuning, bp_waves));' \
          'return 0;}\n' % HEADER
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", c, "-o", os.path.join(d, "s")])
        out = subprocess.check_output([os.path.join(d, "s")]).decode().split()
    assert [int(v) for v in out] == [ctypes.sizeof(GeometryDesc), ctypes.sizeof(Options),
                                      ctypes.sizeof(GeometryInfo), GeometryDesc.im_table.offset,
                                      Options.tol.offset, ctypes.sizeof(Tuning), Tuning.fp_ray_split.offset,
                                      GeometryDesc.allocator.offset, ctypes.sizeof(Allocator),
                                      Tuning.fp_waves_per_pair.offset, Tuning.fp_staged.offset, Tuning.bp_waves.offset]


def _desc(**kw):
    import numpy as np
    from paper_1903_11874_amd.bsgd import GeometryDesc
    d = GeometryDesc()
    angles = np.linspace(0, 3.0, 10)
    base = dict(kind=1, nx=16, ny=16, nz=1, vx=1.0, vy=1.0, vz=1.0, n_views=10, nu=24, nv=1, du=1.0, dv=1.0,
                sod=50.0, sdd=100.0, bx=2, by=2, bz=1, n_row_blocks=2, partition_seed=1, su=1, sv=1, im_mode=0)
    base.update(kw)
    for k, v in base.items():
        setattr(d, k, v)
    d.angles_rad = angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, angles


@pytest.mark.parametrize("bad", [dict(kind=7), dict(nx=0), dict(nz=2), dict(vx=-1.0), dict(n_views=0),
                                 dict(nu=0), dict(du=0.0), dict(sod=200.0), dict(sdd=10.0), dict(bx=17),
                                 dict(n_row_blocks=11), dict(su=25), dict(im_mode=9), dict(sod=9.0, sdd=100.0)])
def test_invalid_descriptors_are_rejected(lib, bad):
    d, keep = _desc(**bad)
    out = ctypes.c_void_p(123)
    st = lib.bsgd_geometry_create(ctypes.byref(d), None, ctypes.byref(out))
    assert st == 1
    assert out.value is None
    assert lib.bsgd_last_error()


def test_allocator_without_free_is_rejected(lib):
    from paper_1903_11874_amd.bsgd import ALLOC_FN, Allocator
    d, keep = _desc()
    a = Allocator()  # free stays NULL
    fn = ALLOC_FN(lambda ctx, n, s: None)
    a.alloc = fn
    d.allocator = ctypes.pointer(a)
    out = ctypes.c_void_p(123)
    assert lib.bsgd_geometry_create(ctypes.byref(d), None, ctypes.byref(out)) == 1
    assert out.value is None


def test_null_arguments(lib):
    assert lib.bsgd_geometry_create(None, None, None) == 1
    assert lib.bsgd_step(None, 1, None) == 1
    assert lib.bsgd_forward_project(None, None, None, None, 0, -1, 0, None) == 1
    assert lib.bsgd_solver_kernel_times(None, None, None) == 1
    lib.bsgd_geometry_destroy(None)
    lib.bsgd_solver_destroy(None)


def test_flag_constants_match_header():
    from paper_1903_11874_amd import bsgd
    text = open(HEADER).read()
    defs = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"#define\s+(BSGD_FLAG_[A-Z_]+)\s+(\d+)", text))
    assert defs == {"BSGD_FLAG_EAGER": bsgd.FLAG_EAGER, "BSGD_FLAG_SUBDET_MEMORY": bsgd.FLAG_SUBDET_MEMORY}
    o = bsgd.make_options(eager=True, subdet_memory=True)
    assert o.flags == bsgd.FLAG_EAGER | bsgd.FLAG_SUBDET_MEMORY
