"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle of the
three-dimensional SIMPLE-TS step (ora3.c).

Only the tests may use this module; the product never imports it.  Arrays are
numpy FP64 in the oracle's layouts: u (nz, ny, nx+1), v (nz, ny+1, nx),
w (nz+1, ny, nx), p and T (nz, ny, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libora3.so")
_lib = None

_D = C.POINTER(C.c_double)

WALLS, PERIODIC, INLET_OUTLET = 0, 1, 2
NOSLIP, SLIP = 0, 1
EXPLICIT, IMPLICIT, UPWIND, TVD = 0, 1, 0, 2
SCHEMES = {"explicit_upwind": EXPLICIT | UPWIND, "explicit_tvd": EXPLICIT | TVD,
           "implicit_upwind": IMPLICIT | UPWIND, "implicit_tvd": IMPLICIT | TVD}


def build(verbose: bool = False) -> str:
    """Compile ora3.c into oracle/libora3.so (plain C, FP64, no FMA contraction)."""
    src = os.path.join(_HERE, "ora3.c")
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", _LIB_PATH + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Setup(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3), ("d", _D * 3), ("bc", C.c_int * 3),
        ("wall_type", (C.c_int * 2) * 3), ("wall_vel", ((C.c_double * 3) * 2) * 3),
        ("wall_T", (C.c_double * 2) * 3),
        ("Ma", C.c_double), ("Re", C.c_double), ("Pr", C.c_double), ("gamma", C.c_double),
        ("u_in", C.c_double), ("T_in", C.c_double), ("p_in", C.c_double),
        ("g", C.c_double * 3),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.ora3_create.restype = C.c_void_p
        L.ora3_create.argtypes = [C.POINTER(_Setup)]
        L.ora3_destroy.argtypes = [C.c_void_p]
        L.ora3_set_threads.argtypes = [C.c_int]
        L.ora3_set_fields.argtypes = [C.c_void_p, _D * 5]
        L.ora3_get_fields.argtypes = [C.c_void_p, _D * 5]
        L.ora3_step.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int]
        L.ora3_residuals.argtypes = [C.c_void_p, _D]
        L.ora3_mass.argtypes = [C.c_void_p]
        L.ora3_mass.restype = C.c_double
        L.ora3_eq_residuals.argtypes = [C.c_void_p, C.c_double, C.c_int, _D * 5]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().ora3_set_threads(int(n))


@dataclass
class Box:
    """A three-dimensional problem: cell widths per direction, the boundary
    kind of each direction, wall data per wall (index [direction][low/high]),
    the nondimensional numbers, the inlet state and the body force."""
    d: tuple                                   # three arrays of cell widths
    bc: tuple = (PERIODIC, WALLS, PERIODIC)
    wall_type: tuple = ((NOSLIP, NOSLIP),) * 3
    wall_vel: tuple = (((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),) * 3
    wall_T: tuple = ((1.0, 1.0),) * 3
    Ma: float = 0.1
    Re: float = 10.0
    Pr: float = 0.7
    gamma: float = 1.4
    u_in: float = 1.0
    T_in: float = 1.0
    p_in: float = 1.0
    g: tuple = (0.0, 0.0, 0.0)
    n: tuple = field(init=False)

    def __post_init__(self):
        self.d = tuple(np.ascontiguousarray(x, dtype=np.float64) for x in self.d)
        self.n = tuple(len(x) for x in self.d)

    def shapes(self):
        nx, ny, nz = self.n
        return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx), (nz, ny, nx)]


class Oracle3:
    """FP64 CPU SIMPLE-TS step in three dimensions on a Box."""

    def __init__(self, box: Box):
        L = lib()
        self.box = box
        s = _Setup()
        for e in range(3):
            s.n[e] = box.n[e]
            s.d[e] = box.d[e].ctypes.data_as(_D)
            s.bc[e] = box.bc[e]
            for w in range(2):
                s.wall_type[e][w] = box.wall_type[e][w]
                s.wall_T[e][w] = box.wall_T[e][w]
                for k in range(3):
                    s.wall_vel[e][w][k] = box.wall_vel[e][w][k]
            s.g[e] = box.g[e]
        s.Ma, s.Re, s.Pr, s.gamma = box.Ma, box.Re, box.Pr, box.gamma
        s.u_in, s.T_in, s.p_in = box.u_in, box.T_in, box.p_in
        self._h = L.ora3_create(C.byref(s))
        if not self._h:
            raise ValueError("ora3_create refused the box (each direction needs >= 4 cells)")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora3_destroy(self._h)
            self._h = None

    def set_fields(self, u=None, v=None, w=None, p=None, T=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                for a in (u, v, w, p, T)]
        for a, shp in zip(arrs, self.box.shapes()):
            if a is not None and a.shape != shp:
                raise ValueError(f"field shape {a.shape}, expected {shp}")
        ptrs = (_D * 5)(*[C.cast(None, _D) if a is None else a.ctypes.data_as(_D) for a in arrs])
        lib().ora3_set_fields(self._h, ptrs)

    def fields(self):
        out = [np.zeros(s) for s in self.box.shapes()]
        lib().ora3_get_fields(self._h, (_D * 5)(*[a.ctypes.data_as(_D) for a in out]))
        return out

    def step(self, dt, n_inner, scheme):
        lib().ora3_step(self._h, float(dt), int(n_inner), int(scheme))

    def residuals(self):
        out = np.zeros(7)
        lib().ora3_residuals(self._h, out.ctypes.data_as(_D))
        return out

    def mass(self):
        return lib().ora3_mass(self._h)

    def eq_residuals(self, dt, scheme):
        """Residuals of every discrete equation at the current state (order
        u, v, w, p, T), the state frozen as both time level n-1 and the old
        iterate."""
        out = [np.zeros(s) for s in self.box.shapes()]
        lib().ora3_eq_residuals(self._h, float(dt), int(scheme),
                                (_D * 5)(*[a.ctypes.data_as(_D) for a in out]))
        return out
