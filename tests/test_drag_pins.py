"""Pins of the oracle's obstacle drag (the loss of the adjoint) by closed
forms: no force in a fluid at rest under uniform pressure, the pressure
drag of a rectangle in a linear pressure field, and the wall shear of a
uniform stream over its top and bottom faces."""
import numpy as np

from paper_1802_04243_amd import workloads as W


def _case():
    p = W.Problem(nx=30, ny=10, lx=3.0, ly=1.0, obstacles=[(10, 3, 14, 6)], Re=25.0, Ma=1.7)
    return p


def _fields(p, u=0.0, pres=None, T=1.0):
    nx, ny = p.nx, p.ny
    uu = np.full((ny, nx + 1), u)
    vv = np.zeros((ny + 1, nx))
    pp = np.ones((ny, nx)) if pres is None else pres
    TT = np.full((ny, nx), T)
    return uu, vv, pp, TT


def test_rest_uniform_pressure_has_no_drag(oracle_lib):
    p = _case()
    assert oracle_lib.drag(p, _fields(p, pres=np.full((p.ny, p.nx), 3.7))) == 0.0


def test_linear_pressure_drag_of_a_rectangle(oracle_lib):
    # p = 1 - g x at the cell centres; the fluid cells west and east of the
    # 5 x 4 block sit 6 cells apart: D = A g (6 dx) (4 dy)
    p = _case()
    g = 0.3
    dx, dy = p.lx / p.nx, p.ly / p.ny
    xc = (np.arange(p.nx) + 0.5) * dx
    pres = np.repeat((1.0 - g * xc)[None, :], p.ny, axis=0)
    A = 1.0 / (p.gamma * p.Ma ** 2)
    d = oracle_lib.drag(p, _fields(p, pres=pres))
    assert abs(d - A * g * 6 * dx * 4 * dy) <= 1e-14


def test_uniform_stream_wall_shear(oracle_lib):
    # the 5 fluid cells above and the 5 below the block each see a wall at
    # half a cell: D = 10 B Gamma U dx / (dy / 2), Gamma = sqrt(T)
    p = _case()
    U, T = 0.8, 1.44
    dx, dy = p.lx / p.nx, p.ly / p.ny
    d = oracle_lib.drag(p, _fields(p, u=U, T=T))
    assert abs(d - 10 * (1.0 / p.Re) * np.sqrt(T) * U * dx / (0.5 * dy)) <= 1e-13
