"""The C-ABI library loads and exports every symbol include/sts.h declares,
and rejects invalid problems before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1802_04243_amd import sts
from paper_1802_04243_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sts.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sts_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(sts.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(sts.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def _create(**kw):
    L = sts.lib()
    nx, ny = kw.get("nx", 16), kw.get("ny", 8)
    g = sts._Grid(nx, ny, kw.get("lx", 1.0), kw.get("ly", 1.0), None, None)
    i0 = np.array([kw.get("i0", 5)], dtype=np.int32)
    j0 = np.array([2], dtype=np.int32)
    i1 = np.array([kw.get("i1", 7)], dtype=np.int32)
    j1 = np.array([4], dtype=np.int32)
    ob = sts._Obst(kw.get("nobs", 1), *[a.ctypes.data_as(sts._I) for a in (i0, j0, i1, j1)])
    bc = sts._Bc()
    bc.x_mode = kw.get("x_mode", 0)
    bc.p_in = kw.get("p_in", 1.0)
    bc.obstacle_T = 1.0
    bc.wall_type[0] = kw.get("wt", 0)
    h = C.c_void_p()
    rc = L.sts_create(C.byref(g), C.byref(ob), kw.get("Ma", 2.0), kw.get("Re", 20.0), 0.7,
                      kw.get("gamma", 1.4), C.byref(bc), None, None, 0, C.byref(h))
    return rc, h, L.sts_last_error().decode()


@pytest.mark.parametrize("kw", [dict(nx=3), dict(ny=2), dict(Ma=0.0), dict(Re=-1.0),
                                dict(gamma=1.0), dict(x_mode=7), dict(wt=5), dict(p_in=0.0),
                                dict(i0=0), dict(i1=15), dict(i0=9, i1=8), dict(lx=0.0),
                                dict(nobs=-1)])
def test_create_rejects_invalid_problems(kw):
    rc, h, msg = _create(**kw)
    assert rc == sts.STS_EINVAL
    assert h.value is None
    assert msg


def test_null_arguments_are_rejected():
    L = sts.lib()
    assert L.sts_step(None, 0.1, 1, 0) == sts.STS_EINVAL
    assert L.sts_residuals(None, None) == sts.STS_EINVAL
    assert L.sts_fields(None, None, None, None, None) == sts.STS_EINVAL
    assert L.sts_workspace_bytes(None, None) == sts.STS_EINVAL
    L.sts_destroy(None)  # NULL-safe


def test_workspace_bytes_scale_with_the_grid():
    L = sts.lib()
    sizes = []
    for n in (64, 128, 256):
        g = sts._Grid(n, n, 1.0, 1.0, None, None)
        b = C.c_size_t()
        assert L.sts_workspace_bytes(C.byref(g), C.byref(b)) == sts.STS_OK
        sizes.append(b.value)
    assert sizes[0] < sizes[1] < sizes[2]
    # 14 FP64 arrays per cell (two states, four step constants, two face
    # mass fluxes) plus framing: about 112 B per finite volume
    assert 112 * 256 * 256 < sizes[2] < 1.3 * 112 * 256 * 256 + 4e5


def declared_functions3():
    text = open(os.path.join(ROOT, "include", "sts3.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sts3_[a-z0-9_]+)\s*\(", text)))


def test_3d_header_matches_binding_and_library():
    from paper_1802_04243_amd import sts3
    assert declared_functions3() == sorted(sts3.EXPORTS3)
    L = C.CDLL(sts.LIB_PATH)
    for name in declared_functions3():
        assert hasattr(L, name), name


def _box3(**kw):
    from paper_1802_04243_amd import workloads3 as W3
    n = kw.pop("n", (8, 6, 5))
    d = kw.pop("d", tuple(np.full(k, 0.1) for k in n))
    return W3.Box3(d=d, **kw)


@pytest.mark.parametrize("kw", [dict(n=(3, 6, 5)), dict(n=(8, 6, 3)),
                                dict(d=(np.full(8, 0.1), np.full(6, -0.1), np.full(5, 0.1))),
                                dict(bc=(0, 0, 0)), dict(bc=(1, 2, 0)), dict(Ma=0.0),
                                dict(Re=-1.0), dict(gamma=1.0), dict(p_in=0.0), dict(T_in=0.0),
                                dict(wall_type=((0, 0), (3, 0), (0, 0))),
                                dict(wall_T=((1, 1), (0.0, 1), (1, 1)))])
def test_3d_create_rejects_invalid_setups(kw):
    from paper_1802_04243_amd import sts3
    box = _box3(**kw)
    h = C.c_void_p()
    rc = sts3.lib3().sts3_create(C.byref(sts3.setup_of(box)), None, C.byref(h))
    assert rc == sts.STS_EINVAL
    assert h.value is None
    assert sts.lib().sts_last_error().decode()


def test_3d_null_arguments_and_device_bytes():
    from paper_1802_04243_amd import sts3
    L = sts3.lib3()
    assert L.sts3_step(None, 0.1, 1, 0) == sts.STS_EINVAL
    assert L.sts3_residuals(None, None) == sts.STS_EINVAL
    assert L.sts3_create(None, None, None) == sts.STS_EINVAL
    L.sts3_destroy(None)
    b = C.c_size_t()
    assert L.sts3_device_bytes((C.c_int * 3)(64, 32, 32), C.byref(b)) == sts.STS_OK
    # 29 FP64 arrays of (nz+1+4) (ny+1+4) rows of a pitch of 96 doubles for
    # nx = 64 (two ghost layers at each end of every direction)
    assert b.value == 29 * 8 * 96 * 37 * 37
    assert L.sts3_device_bytes((C.c_int * 3)(64, 3, 32), C.byref(b)) == sts.STS_EINVAL
