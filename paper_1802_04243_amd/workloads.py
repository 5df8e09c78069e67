"""Seeded synthetic workloads for the SIMPLE-TS solver.

This module only describes inputs: grid sizes, channel geometry, square
obstacles (as closed cell-index rectangles), gas parameters, boundary values
and the seeded initial noise.  It holds none of the solver's arithmetic, so
both the HIP library and the CPU oracle can be fed from it.

Geometry follows the test case of the paper (Sec. 4, flow past squares in a
channel), restated in convective units: channel height H = 1, length 5H,
supersonic inlet u = 1, T = p = 1 at x = 0, zero-gradient outlet, no-slip
isothermal walls at the inlet temperature, squares of side H/4 centred at
y = H/2.  The time step is dt = min(0.2 h / U_in, 0.5 Re h^2) with h = min(dx, dy).
"""
from __future__ import annotations

import dataclasses
import math
from fractions import Fraction
from typing import List, Optional, Sequence, Tuple

import numpy as np

EXPLICIT, IMPLICIT = 0, 1
UPWIND, TVD = 0, 2
MIXED = 4  # mixed-precision form of any of the four variants
SCHEMES = {
    "explicit_upwind": EXPLICIT | UPWIND,
    "explicit_tvd": EXPLICIT | TVD,
    "implicit_upwind": IMPLICIT | UPWIND,
    "implicit_tvd": IMPLICIT | TVD,
}
WALL_NOSLIP_ISOTHERMAL, WALL_SLIP_ADIABATIC, WALL_SLIP_JUMP = 0, 1, 2


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    lx: float = 5.0
    ly: float = 1.0
    dx: Optional[np.ndarray] = None          # [nx] widths; uniform if None
    dy: Optional[np.ndarray] = None          # [ny]
    periodic: bool = False
    obstacles: List[Tuple[int, int, int, int]] = dataclasses.field(default_factory=list)  # (i0, j0, i1, j1) closed
    Ma: float = 2.43
    Re: float = 20.0
    Pr: float = 0.70
    gamma: float = 1.4
    u_in: Optional[np.ndarray] = None        # [ny]
    T_in: Optional[np.ndarray] = None        # [ny]
    p_in: float = 1.0
    wall_type: Tuple[int, int] = (WALL_NOSLIP_ISOTHERMAL, WALL_NOSLIP_ISOTHERMAL)
    wall_u: Tuple[float, float] = (0.0, 0.0)
    wall_T: Tuple[Optional[np.ndarray], Optional[np.ndarray]] = (None, None)  # [nx] each
    obstacle_T: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    obstacle_type: int = WALL_NOSLIP_ISOTHERMAL  # or WALL_SLIP_JUMP
    kn: float = 0.0                              # Knudsen number of slip / jump surfaces

    def widths(self) -> Tuple[np.ndarray, np.ndarray]:
        dx = self.dx if self.dx is not None else np.full(self.nx, self.lx / self.nx)
        dy = self.dy if self.dy is not None else np.full(self.ny, self.ly / self.ny)
        return np.ascontiguousarray(dx, dtype=np.float64), np.ascontiguousarray(dy, dtype=np.float64)

    def inlet(self) -> Tuple[np.ndarray, np.ndarray]:
        u = self.u_in if self.u_in is not None else np.ones(self.ny)
        t = self.T_in if self.T_in is not None else np.ones(self.ny)
        return np.ascontiguousarray(u, dtype=np.float64), np.ascontiguousarray(t, dtype=np.float64)

    def walls(self) -> Tuple[np.ndarray, np.ndarray]:
        out = []
        for w in self.wall_T:
            out.append(np.ascontiguousarray(w if w is not None else np.ones(self.nx), dtype=np.float64))
        return out[0], out[1]

    def solid_mask(self) -> np.ndarray:
        """Cell mask of the obstacle rectangles (1 = solid), shape (ny, nx)."""
        m = np.zeros((self.ny, self.nx), dtype=np.uint8)
        for i0, j0, i1, j1 in self.obstacles:
            m[j0:j1 + 1, i0:i1 + 1] = 1
        return m

    def cfl_dt(self, cfl: float = 0.2, sigma: float = 0.5) -> float:
        """Time step of the workloads: dt = min(cfl h / U_in, sigma Re h^2), h = min(dx, dy).

        The inner Jacobi loop of the method converges only for a bounded convective
        Courant number and a bounded viscous number B dt / h^2 (B = 1/Re); both limits
        are applied.
        """
        dx, dy = self.widths()
        h = min(float(dx.min()), float(dy.min()))
        umax = float(np.max(np.abs(self.inlet()[0]))) if not self.periodic else 1.0
        return min(cfl * h / max(umax, 1e-300), sigma * self.Re * h * h)

    @property
    def n_fv(self) -> int:
        return self.nx * self.ny


# ---------------------------------------------------------------------------
# geometry helpers (exact rational arithmetic: no rounding decides a cell)
# ---------------------------------------------------------------------------
def square_cells(nx: int, ny: int, lx: Fraction, ly: Fraction, xc: Fraction, yc: Fraction,
                 side: Fraction) -> Tuple[int, int, int, int]:
    """Closed index rectangle of the cells whose centres lie in the square."""
    dx, dy = lx / nx, ly / ny
    x0, x1 = xc - side / 2, xc + side / 2
    y0, y1 = yc - side / 2, yc + side / 2
    i0 = math.ceil(x0 / dx - Fraction(1, 2))
    i1 = math.floor(x1 / dx - Fraction(1, 2))
    j0 = math.ceil(y0 / dy - Fraction(1, 2))
    j1 = math.floor(y1 / dy - Fraction(1, 2))
    return (max(i0, 0), max(j0, 0), min(i1, nx - 1), min(j1, ny - 1))


def channel(nx: int, ny: int, centres: Sequence[Fraction], Re: float = 20.0, **kw) -> Problem:
    """Channel 5H x H with squares of side H/4 centred at (xc, H/2)."""
    lx, ly = Fraction(5), Fraction(1)
    obst = [square_cells(nx, ny, lx, ly, Fraction(xc), Fraction(1, 2), Fraction(1, 4)) for xc in centres]
    return Problem(nx=nx, ny=ny, lx=5.0, ly=1.0, obstacles=obst, Re=Re, **kw)


def paper_channel(ny: int, kn: float = 0.001, Ma: float = 2.43) -> Problem:
    """The test case of Sec. 4 in the paper's own units (length: the square
    side a; velocity: the thermal speed V_th = sqrt(2 R T_0); T_0 the wall
    temperature, p_0 the inflow pressure): uniform grid spacing 0.05, channel
    length 201.6 (4032 cells), height ny * 0.05, one square of side 1 whose
    front face is 5.5 behind the inlet, centred in y; hard-sphere gas with
    gamma = 5/3, Pr = 2/3 and the pl37 coefficients (A = 1/2,
    B = 5 sqrt(pi) Kn / 16), i.e. a reference Mach number sqrt(2/gamma) and a
    reference Reynolds number 16 / (5 sqrt(pi) Kn); inflow at Mach Ma, i.e.
    u = Ma sqrt(gamma/2) in V_th units; particle frame: the channel walls move
    with the inflow speed; velocity-slip / temperature-jump walls and square
    (pl38, pl39) at T = 1."""
    nx, d = 4032, 0.05
    gamma = 5.0 / 3.0
    U = Ma * math.sqrt(gamma / 2.0)
    i0 = 110                           # 5.5 / 0.05
    j0 = ny // 2 - 10
    return Problem(nx=nx, ny=ny, lx=nx * d, ly=ny * d, obstacles=[(i0, j0, i0 + 19, j0 + 19)],
                   Ma=math.sqrt(2.0 / gamma), Re=16.0 / (5.0 * math.sqrt(math.pi) * kn),
                   Pr=2.0 / 3.0, gamma=gamma, u_in=np.full(ny, U),
                   wall_type=(WALL_SLIP_JUMP, WALL_SLIP_JUMP), wall_u=(U, U),
                   obstacle_type=WALL_SLIP_JUMP, kn=kn)


# named workloads ------------------------------------------------------------
def workload(name: str) -> Tuple[Problem, dict]:
    """Problem plus run parameters (steps, inner iterations, dt, seed)."""
    h = Fraction(1)
    if name == "channel_120x24":          # small case: one centred square, 50 steps x 20 inner
        p = channel(120, 24, [Fraction(5, 2) * h])
        run = dict(steps=50, inner=20, seed=1)
    elif name == "channel_1280x288":      # mid size, two squares
        p = channel(1280, 288, [Fraction(3, 2), Fraction(3)])
        run = dict(steps=200, inner=10, seed=3)
    elif name == "channel_3000x600":      # 1.8M FV, two squares at 1.5H and 3H
        p = channel(3000, 600, [Fraction(3, 2), Fraction(3)])
        run = dict(steps=200, inner=10, seed=2)
    elif name == "channel_5120x1152":     # 5.9M FV, two squares at 1.5H and 3H
        p = channel(5120, 1152, [Fraction(3, 2), Fraction(3)])
        run = dict(steps=200, inner=10, seed=3)
    elif name == "channel_1024x256":      # one square centred
        p = channel(1024, 256, [Fraction(5, 2)])
        run = dict(steps=100, inner=10, seed=4)
    elif name == "adjoint_1024x256":      # one square centred, parabolic seeded inlet
        p = channel(1024, 256, [Fraction(5, 2)], u_in=parabolic_inlet(256, 4))
        run = dict(steps=100, inner=10, seed=4, every=10)
    elif name == "channel_4096x1024":     # two squares, Re 50
        p = channel(4096, 1024, [Fraction(3, 2), Fraction(3)], Re=50.0)
        run = dict(steps=500, inner=10, seed=5)
    elif name == "combined_4096x1024":    # mixed forward + FP64 adjoint, sqrt(N) checkpoints
        p = channel(4096, 1024, [Fraction(3, 2), Fraction(3)], Re=50.0)
        run = dict(steps=500, inner=10, seed=5, every=None)
    elif name.startswith("paper_4032x") and name[len("paper_4032x"):] in ("200", "400", "2000", "4000"):
        # the paper's meshes (Sec. 4): channel heights 10, 20, 100, 200
        p = paper_channel(int(name[len("paper_4032x"):]))
        # Courant number 0.1 of the inflow speed: at 0.2 the explicit TVD
        # scheme's loop 2 diverges on this supersonic flow (its last-pass
        # increments grow to non-finite values within 200 steps); at 0.1 they
        # stay below 1e-6 over 200 steps in every scheme
        run = dict(steps=200, inner=10, seed=6, cfl=0.1)
    else:
        raise KeyError(name)
    run["dt"] = p.cfl_dt(**({"cfl": run.pop("cfl")} if "cfl" in run else {}))
    return p, run


# ---------------------------------------------------------------------------
# seeded noise: SplitMix64, one draw per array element
# ---------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n consecutive SplitMix64 outputs of the stream `seed`, starting at draw `offset`."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1): (x >> 11) * 2^-53."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def parabolic_inlet(ny: int, seed: int, amp: float = 1e-2) -> np.ndarray:
    """Inlet profile 4 y (1 - y) (peak 1 at mid-height, cell-centre y in units
    of H) plus a seeded perturbation amp (2U - 1) per row."""
    y = (np.arange(ny) + 0.5) / ny
    return 4.0 * y * (1.0 - y) + amp * (2.0 * uniform01(seed ^ 0x5A5A, ny) - 1.0)


def initial_fields(p: Problem, seed: int, amp: float = 1e-3):
    """Uniform inlet state plus additive noise amp*(2U-1) on u, v and T.

    Draw order: every element of u, then v, then T, rows outer, x inner.
    Boundary values (walls, inlet, solid cells) are imposed by the solver
    that receives the fields.
    """
    nx, ny = p.nx, p.ny
    u_in, T_in = p.inlet()
    nu, nv, nc = (nx + 1) * ny, nx * (ny + 1), nx * ny
    r = uniform01(seed, nu + nv + nc)
    u = np.repeat(u_in[:, None], nx + 1, axis=1) + amp * (2 * r[:nu].reshape(ny, nx + 1) - 1)
    v = amp * (2 * r[nu:nu + nv].reshape(ny + 1, nx) - 1)
    T = np.repeat(T_in[:, None], nx, axis=1) + amp * (2 * r[nu + nv:].reshape(ny, nx) - 1)
    pr = np.full((ny, nx), p.p_in)
    return (np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(pr),
            np.ascontiguousarray(T))
