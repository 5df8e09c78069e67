"""ctypes binding of libsts.so (the C ABI in include/sts.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch, when present, supplies the device workspace and the HIP
stream the library enqueues on.  If the library is missing the binding raises;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsts.so")

STS_OK, STS_EINVAL, STS_ENOMEM, STS_EDEVICE, STS_ENONFINITE, STS_ESTATE = 0, -1, -2, -3, -4, -5
EXPLICIT, IMPLICIT, UPWIND, TVD, MIXED = 0, 1, 0, 2, 4

# every symbol the header declares
EXPORTS = ("sts_workspace_bytes", "sts_create", "sts_step", "sts_step_tol", "sts_residuals",
           "sts_residual_history", "sts_fields",
           "sts_set_fields", "sts_field_ptrs", "sts_timing", "sts_read_timing", "sts_drag", "sts_drag_noalloc",
           "sts_state_slots", "sts_state_save", "sts_state_load", "sts_adjoint_begin",
           "sts_adjoint_seed_drag", "sts_adjoint_seed", "sts_adjoint_step", "sts_step_l3", "sts_step_tol_l3", "sts_adjoint_read", "sts_adjoint_read_state_grad", "sts_destroy",
           "sts_last_error")

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


class StsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sts error {code}: {msg}")
        self.code = code


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("lx", C.c_double), ("ly", C.c_double),
                ("dx", _D), ("dy", _D)]


class _Obst(C.Structure):
    _fields_ = [("n", C.c_int), ("i0", _I), ("j0", _I), ("i1", _I), ("j1", _I)]


class _Bc(C.Structure):
    _fields_ = [("x_mode", C.c_int), ("u_in", _D), ("T_in", _D), ("p_in", C.c_double),
                ("wall_type", C.c_int * 2), ("wall_u", C.c_double * 2), ("wall_T", _D * 2),
                ("obstacle_T", C.c_double), ("gx", C.c_double), ("gy", C.c_double),
                ("obstacle_type", C.c_int), ("kn", C.c_double)]


_lib = None


def lib():
    """Load libsts.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1802_04243_amd/build.py")
        try:  # bind to the HIP runtime torch already loaded, if any
            import torch  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(LIB_PATH)
        L.sts_workspace_bytes.argtypes = [C.POINTER(_Grid), C.POINTER(C.c_size_t)]
        L.sts_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Obst), C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.POINTER(_Bc), C.c_void_p, C.c_void_p,
                                 C.c_size_t, C.POINTER(C.c_void_p)]
        L.sts_step.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int]
        L.sts_step_tol.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_int,
                                   C.POINTER(C.c_int)]
        L.sts_residuals.argtypes = [C.c_void_p, _D]
        L.sts_residual_history.argtypes = [C.c_void_p, _D, C.c_int, C.POINTER(C.c_int)]
        L.sts_fields.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.sts_set_fields.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.sts_field_ptrs.argtypes = [C.c_void_p] + [C.POINTER(C.c_void_p)] * 4 + \
            [C.POINTER(C.c_size_t)] * 2
        L.sts_timing.argtypes = [C.c_void_p, C.c_int]
        L.sts_read_timing.argtypes = [C.c_void_p, _D, C.POINTER(C.c_longlong)]
        L.sts_drag.argtypes = [C.c_void_p, _D]
        L.sts_drag_noalloc.argtypes = [C.c_void_p, C.c_void_p]
        L.sts_state_slots.argtypes = [C.c_void_p, C.c_int]
        L.sts_state_save.argtypes = [C.c_void_p, C.c_int]
        L.sts_state_load.argtypes = [C.c_void_p, C.c_int]
        L.sts_adjoint_begin.argtypes = [C.c_void_p, C.c_int]
        L.sts_adjoint_seed_drag.argtypes = [C.c_void_p, C.c_double]
        L.sts_adjoint_seed.argtypes = [C.c_void_p] + [_D] * 4
        L.sts_step_l3.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_int]
        L.sts_step_tol_l3.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_double,
                                      C.c_int, C.POINTER(C.c_int)]
        L.sts_adjoint_step.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int]
        L.sts_adjoint_read.argtypes = [C.c_void_p] + [_D] * 7
        L.sts_adjoint_read_state_grad.argtypes = [C.c_void_p] + [_D] * 4
        L.sts_destroy.argtypes = [C.c_void_p]
        L.sts_destroy.restype = None
        L.sts_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("sts_destroy", "sts_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != STS_OK:
        raise StsError(code, lib().sts_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


class Solver:
    """One SIMPLE-TS solver on the current HIP device.

    use_torch: take the workspace from torch (device memory) and enqueue on
    torch's current stream; otherwise the library allocates and owns a stream.
    """

    def __init__(self, prob: W.Problem, use_torch: bool = True):
        L = lib()
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        dx, dy = prob.widths()
        u_in, T_in = prob.inlet()
        wb, wt = prob.walls()
        ob = np.array(prob.obstacles, dtype=np.int32).reshape(-1, 4)
        cols = [np.ascontiguousarray(ob[:, k]) for k in range(4)]
        self._keep = [dx, dy, u_in, T_in, wb, wt, *cols]
        g = _Grid(prob.nx, prob.ny, prob.lx, prob.ly, _ptr(dx), _ptr(dy))
        o = _Obst(len(ob), *[c.ctypes.data_as(_I) for c in cols])
        bc = _Bc()
        bc.x_mode = 1 if prob.periodic else 0
        bc.u_in, bc.T_in, bc.p_in = _ptr(u_in), _ptr(T_in), prob.p_in
        bc.wall_type[0], bc.wall_type[1] = prob.wall_type
        bc.wall_u[0], bc.wall_u[1] = prob.wall_u
        bc.wall_T[0], bc.wall_T[1] = _ptr(wb), _ptr(wt)
        bc.obstacle_T, bc.gx, bc.gy = prob.obstacle_T, prob.gx, prob.gy
        bc.obstacle_type, bc.kn = prob.obstacle_type, prob.kn
        nbytes = C.c_size_t()
        _check(L.sts_workspace_bytes(C.byref(g), C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        stream, ws = None, None
        self._ws = None
        if use_torch:
            import torch
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ws = (base + 255) // 256 * 256
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(L.sts_create(C.byref(g), C.byref(o), prob.Ma, prob.Re, prob.Pr, prob.gamma,
                            C.byref(bc), stream, ws, nbytes.value, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sts_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self):
        nx, ny = self.nx, self.ny
        return (ny, nx + 1), (ny + 1, nx), (ny, nx), (ny, nx)

    def step(self, dt: float, n_inner: int, scheme: int):
        _check(lib().sts_step(self._h, float(dt), int(n_inner), int(scheme)))

    def step_l3(self, dt: float, n_inner: int, n3: int, scheme: int):
        """One step whose passes each solve the energy and pressure equations n3 times."""
        _check(lib().sts_step_l3(self._h, float(dt), int(n_inner), int(n3), int(scheme)))

    def step_tol_l3(self, dt: float, max_inner: int, n3: int, tol: float, scheme: int) -> int:
        """step_tol with loop 3 (n3 energy-pressure solves) in every pass."""
        n = C.c_int(0)
        _check(lib().sts_step_tol_l3(self._h, float(dt), int(max_inner), int(n3), float(tol),
                                     int(scheme), C.byref(n)))
        return n.value

    def step_tol(self, dt: float, max_inner: int, tol: float, scheme: int) -> int:
        """One step with loop 2 stopped at the tolerance; returns the passes taken."""
        n = C.c_int(0)
        _check(lib().sts_step_tol(self._h, float(dt), int(max_inner), float(tol), int(scheme),
                                  C.byref(n)))
        return n.value

    def residuals(self) -> np.ndarray:
        out = np.zeros(6)
        _check(lib().sts_residuals(self._h, _ptr(out)))
        return out

    def residual_history(self) -> np.ndarray:
        """Per-pass max|du|, max|dv|, max|dp|, max|dT| of the last tolerance
        step, shape (passes, 4)."""
        rows = C.c_int(0)
        _check(lib().sts_residual_history(self._h, None, 0, C.byref(rows)))
        out = np.zeros((rows.value, 4))
        if rows.value:
            _check(lib().sts_residual_history(self._h, _ptr(out), rows.value, C.byref(rows)))
        return out

    def fields(self) -> Tuple[np.ndarray, ...]:
        out = [np.zeros(s) for s in self.shapes()]
        _check(lib().sts_fields(self._h, *[_ptr(a) for a in out]))
        return tuple(out)

    def set_fields(self, u=None, v=None, p=None, T=None):
        arrs = []
        for a, shp in zip((u, v, p, T), self.shapes()):
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != shp:
                    raise ValueError(f"field shape {a.shape}, expected {shp}")
            arrs.append(a)
        _check(lib().sts_set_fields(self._h, *[_ptr(a) for a in arrs]))

    def field_ptrs(self):
        ptrs = [C.c_void_p() for _ in range(4)]
        origin, pitch = C.c_size_t(), C.c_size_t()
        _check(lib().sts_field_ptrs(self._h, *[C.byref(p) for p in ptrs], C.byref(origin),
                                    C.byref(pitch)))
        return [p.value for p in ptrs], origin.value, pitch.value

    def timing(self, enable: bool = True):
        _check(lib().sts_timing(self._h, int(enable)))

    def read_timing(self):
        ms = np.zeros(3)
        n = (C.c_longlong * 2)()
        _check(lib().sts_read_timing(self._h, _ptr(ms), n))
        return ms, (n[0], n[1])

    # ---- loss, checkpoints, adjoint of the explicit step ----
    def drag(self) -> float:
        out = np.zeros(1)
        _check(lib().sts_drag(self._h, _ptr(out)))
        return float(out[0])

    def drag_noalloc(self, out) -> None:
        """sts_drag_noalloc: enqueue the drag into out[0], a float64 tensor on
        the solver's GPU (no allocation, no wait)."""
        assert out.is_cuda and out.dtype.is_floating_point and out.element_size() == 8
        _check(lib().sts_drag_noalloc(self._h, C.c_void_p(out.data_ptr())))

    def state_slots(self, n: int):
        _check(lib().sts_state_slots(self._h, int(n)))

    def state_save(self, slot: int):
        _check(lib().sts_state_save(self._h, int(slot)))

    def state_load(self, slot: int):
        _check(lib().sts_state_load(self._h, int(slot)))

    def adjoint_begin(self, n_inner: int):
        _check(lib().sts_adjoint_begin(self._h, int(n_inner)))

    def adjoint_seed_drag(self, w: float):
        _check(lib().sts_adjoint_seed_drag(self._h, float(w)))

    def adjoint_seed(self, lu=None, lv=None, lp=None, lT=None):
        """lambda += the given arrays (field shapes; None skips a field)."""
        arrs = []
        for a, shp in zip((lu, lv, lp, lT), self.shapes()):
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != shp:
                    raise ValueError(f"seed shape {a.shape}, expected {shp}")
            arrs.append(a)
        _check(lib().sts_adjoint_seed(self._h, *[_ptr(a) for a in arrs]))

    def adjoint_step(self, dt: float, n_inner: int, scheme: int):
        _check(lib().sts_adjoint_step(self._h, float(dt), int(n_inner), int(scheme)))

    def adjoint_state_grad(self):
        """dL/d(the fields given to set_fields at the current level), layouts
        of fields() (sts_adjoint_read_state_grad)."""
        out = [np.zeros(s) for s in self.shapes()]
        _check(lib().sts_adjoint_read_state_grad(self._h, *[_ptr(a) for a in out]))
        return tuple(out)

    def adjoint_read(self, with_lambda: bool = False):
        """(dL/du_in[ny], dL/dwall_T[0][nx], dL/dwall_T[1][nx]) and, if asked,
        the adjoint state (u, v, p, T layouts of fields())."""
        g = [np.zeros(self.ny), np.zeros(self.nx), np.zeros(self.nx)]
        lam = [np.zeros(s) for s in self.shapes()] if with_lambda else [None] * 4
        _check(lib().sts_adjoint_read(self._h, *[_ptr(a) for a in g], *[_ptr(a) for a in lam]))
        return (tuple(g), tuple(lam)) if with_lambda else tuple(g)
