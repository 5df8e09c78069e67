"""ctypes binding of the three-dimensional step in libsts.so (include/sts3.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch, when present, supplies the HIP stream the library enqueues
on.  If the library is missing the binding raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import sts as S
from .workloads3 import Box3

EXPORTS3 = ("sts3_create", "sts3_device_bytes", "sts3_step", "sts3_residuals", "sts3_fields",
            "sts3_set_fields", "sts3_destroy")

_D = C.POINTER(C.c_double)
_lib3 = None


class _Setup3(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3), ("d", _D * 3), ("bc", C.c_int * 3),
        ("wall_type", (C.c_int * 2) * 3), ("wall_vel", ((C.c_double * 3) * 2) * 3),
        ("wall_T", (C.c_double * 2) * 3),
        ("Ma", C.c_double), ("Re", C.c_double), ("Pr", C.c_double), ("gamma", C.c_double),
        ("u_in", C.c_double), ("T_in", C.c_double), ("p_in", C.c_double),
        ("g", C.c_double * 3),
    ]


def lib3():
    global _lib3
    if _lib3 is None:
        L = S.lib()
        L.sts3_create.argtypes = [C.POINTER(_Setup3), C.c_void_p, C.POINTER(C.c_void_p)]
        L.sts3_device_bytes.argtypes = [C.c_int * 3, C.POINTER(C.c_size_t)]
        L.sts3_step.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int]
        L.sts3_residuals.argtypes = [C.c_void_p, _D]
        L.sts3_fields.argtypes = [C.c_void_p, _D * 5]
        L.sts3_set_fields.argtypes = [C.c_void_p, _D * 5]
        L.sts3_destroy.argtypes = [C.c_void_p]
        L.sts3_destroy.restype = None
        for name in EXPORTS3:
            if name != "sts3_destroy":
                getattr(L, name).restype = C.c_int
        _lib3 = L
    return _lib3


def setup_of(box: Box3) -> _Setup3:
    s = _Setup3()
    for e in range(3):
        s.n[e] = box.n[e]
        s.d[e] = box.d[e].ctypes.data_as(_D)
        s.bc[e] = box.bc[e]
        s.g[e] = box.g[e]
        for w in range(2):
            s.wall_type[e][w] = box.wall_type[e][w]
            s.wall_T[e][w] = box.wall_T[e][w]
            for k in range(3):
                s.wall_vel[e][w][k] = box.wall_vel[e][w][k]
    s.Ma, s.Re, s.Pr, s.gamma = box.Ma, box.Re, box.Pr, box.gamma
    s.u_in, s.T_in, s.p_in = box.u_in, box.T_in, box.p_in
    return s


class Solver3:
    """One 3-D SIMPLE-TS solver on the current HIP device, enqueued on torch's
    current stream (use_torch) or on a stream the library owns."""

    def __init__(self, box: Box3, use_torch: bool = True):
        self.box = box
        stream = None
        if use_torch:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        S._check(lib3().sts3_create(C.byref(setup_of(box)), stream, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib3().sts3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt: float, n_inner: int, scheme: int):
        S._check(lib3().sts3_step(self._h, float(dt), int(n_inner), int(scheme)))

    def residuals(self) -> np.ndarray:
        out = np.zeros(7)
        S._check(lib3().sts3_residuals(self._h, out.ctypes.data_as(_D)))
        return out

    def fields(self):
        out = [np.zeros(s) for s in self.box.shapes()]
        S._check(lib3().sts3_fields(self._h, (_D * 5)(*[a.ctypes.data_as(_D) for a in out])))
        return out

    def set_fields(self, u=None, v=None, w=None, p=None, T=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                for a in (u, v, w, p, T)]
        for a, shp in zip(arrs, self.box.shapes()):
            if a is not None and a.shape != shp:
                raise ValueError(f"field shape {a.shape}, expected {shp}")
        ptrs = (_D * 5)(*[C.cast(None, _D) if a is None else a.ctypes.data_as(_D) for a in arrs])
        S._check(lib3().sts3_set_fields(self._h, ptrs))
