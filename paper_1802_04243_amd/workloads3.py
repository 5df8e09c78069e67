"""Three-dimensional problems and seeded inputs (no method arithmetic).

A Box3 describes a staggered Cartesian grid in x, y, z with its boundary
kinds, wall data, gas and flow parameters; the named workloads are ducts
(supersonic inlet and zero-gradient outlet in x, no-slip isothermal walls in
y and z: the 2-D channel of the paper's test case with a square cross
section, without the obstacle) and periodic boxes.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np

from .workloads import uniform01

WALLS, PERIODIC, INLET_OUTLET = 0, 1, 2
NOSLIP, SLIP = 0, 1


@dataclasses.dataclass
class Box3:
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
    n: tuple = dataclasses.field(init=False)

    def __post_init__(self):
        self.d = tuple(np.ascontiguousarray(x, dtype=np.float64) for x in self.d)
        self.n = tuple(len(x) for x in self.d)

    def shapes(self):
        """Host array shapes of u, v, w, p, T (x fastest)."""
        nx, ny, nz = self.n
        return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx), (nz, ny, nx)]

    @property
    def n_fv(self) -> int:
        return int(np.prod(self.n))

    def cfl_dt(self, cfl: float = 0.2, sigma: float = 0.3) -> float:
        """dt = min(cfl h / U, sigma Re h^2), h the smallest width, U the inlet
        speed (1 in a periodic box): the 2-D workloads' rule with the viscous
        number lowered for the third direction's diffusion."""
        h = min(float(x.min()) for x in self.d)
        u = abs(self.u_in) if self.bc[0] == INLET_OUTLET else 1.0
        return min(cfl * h / max(u, 1e-300), sigma * self.Re * h * h)


def duct(nx: int, ny: int, nz: int, Ma: float = 2.43, Re: float = 20.0, **kw) -> Box3:
    """Duct 5H x H x H: supersonic inlet at x = 0 (u = 1, T = 1, p = 1),
    zero-gradient outlet, no-slip isothermal walls (T = 1) in y and z."""
    return Box3(d=(np.full(nx, 5.0 / nx), np.full(ny, 1.0 / ny), np.full(nz, 1.0 / nz)),
                bc=(INLET_OUTLET, WALLS, WALLS), Ma=Ma, Re=Re, **kw)


def workload3(name: str) -> Tuple[Box3, dict]:
    """Problem plus run parameters (steps, inner iterations, dt, seed)."""
    if name == "duct_60x12x12":        # small case (8.6K FV)
        b = duct(60, 12, 12)
        run = dict(steps=20, inner=10, seed=11)
    elif name == "duct_160x32x32":     # mid size (164K FV)
        b = duct(160, 32, 32)
        run = dict(steps=50, inner=10, seed=12)
    elif name == "duct_512x128x128":   # 8.4M FV
        b = duct(512, 128, 128)
        run = dict(steps=20, inner=10, seed=13)
    else:
        raise KeyError(name)
    run["dt"] = b.cfl_dt()
    return b, run


def initial_fields3(b: Box3, seed: int, amp: float = 1e-3):
    """Uniform inlet state (rest in a periodic x) plus additive noise
    amp*(2U-1) on u, v, w and T; draw order u, v, w, T, x fastest.  Boundary
    values are imposed by the solver that receives the fields."""
    shp = b.shapes()
    sizes = [int(np.prod(s)) for s in shp]
    r = uniform01(seed, sizes[0] + sizes[1] + sizes[2] + sizes[4])
    o = np.cumsum([0, sizes[0], sizes[1], sizes[2]])
    u0 = b.u_in if b.bc[0] == INLET_OUTLET else 0.0
    u = u0 + amp * (2 * r[o[0]:o[1]].reshape(shp[0]) - 1)
    v = amp * (2 * r[o[1]:o[2]].reshape(shp[1]) - 1)
    w = amp * (2 * r[o[2]:o[3]].reshape(shp[2]) - 1)
    T = b.T_in + amp * (2 * r[o[3]:].reshape(shp[4]) - 1)
    p = np.full(shp[3], b.p_in)
    return [np.ascontiguousarray(a) for a in (u, v, w, p, T)]
