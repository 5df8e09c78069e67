"""Pins of the three-dimensional FP64 oracle (oracle/ora3.c) against what the
mathematics and the pinned two-dimensional oracle fix.

The paper states the method in two dimensions (Sec. 3.2) and names 3-D flow
as the next step (Conclusions).  The 3-D oracle reads every 2-D formula per
pair of directions; these tests hold it to:
  - bitwise free-stream preservation (every scheme, periodic box and
    inlet/outlet channel);
  - a flow that does not depend on z (w = 0, z periodic): every x/y equation
    equals the 2-D oracle's, and time steps with loop 2 converged give the
    2-D oracle's fields; this carries the 2-D pins (manufactured solutions,
    Couette, Poiseuille) over to every x/y term;
  - exchanging two axes commutes with every discrete equation: the terms in
    z are the x/y terms with the directions renamed;
  - compressible Couette flow between walls moving in an oblique direction
    (closed form, second order), between y walls and between z walls;
  - mass conservation of converged passes in a closed box.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import oracle3 as O3
from paper_1802_04243_amd import workloads as W
from test_oracle_pins import _couette_exact


@pytest.fixture(scope="module", autouse=True)
def _one_thread():
    # these grids are small: one thread; the OpenMP setting is per process
    # (both oracles share it), so it is restored for the modules that follow
    prev = O.max_threads()
    O3.set_threads(1)
    yield
    O3.set_threads(prev)


def _ones(box):
    return [np.ones(s) for s in box.shapes()]


# ---------------------------------------------------------------------------
# free stream
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", list(O3.SCHEMES.values()))
@pytest.mark.parametrize("kind", ["periodic_diagonal", "channel"])
def test_free_stream_is_preserved_bitwise(scheme, kind):
    rng = np.random.default_rng(3)
    d = (rng.uniform(0.05, 0.15, 8), rng.uniform(0.05, 0.15, 6), rng.uniform(0.05, 0.15, 5))
    if kind == "periodic_diagonal":
        box = O3.Box(d=d, bc=(O3.PERIODIC,) * 3)
        f = _ones(box)  # (u, v, w) = (1, 1, 1), p = T = 1
    else:
        box = O3.Box(d=d, bc=(O3.INLET_OUTLET, O3.WALLS, O3.WALLS),
                     wall_type=((O3.SLIP, O3.SLIP),) * 3)
        f = _ones(box)
        f[1][:] = 0.0
        f[2][:] = 0.0
    o = O3.Oracle3(box)
    o.set_fields(*f)
    f0 = o.fields()
    for _ in range(6):
        o.step(0.01, 5, scheme)
    for a, b in zip(o.fields(), f0):
        assert np.array_equal(a, b)
    assert np.all(o.residuals() == 0.0)


# ---------------------------------------------------------------------------
# a z-invariant flow is the 2-D oracle's flow
# ---------------------------------------------------------------------------
def _pair(periodic, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 14, 9, 4
    dx, dy, dz = rng.uniform(0.05, 0.2, nx), rng.uniform(0.05, 0.2, ny), np.full(nz, 0.13)
    p = W.Problem(nx=nx, ny=ny, dx=dx, dy=dy, periodic=periodic, gx=0.3, gy=-0.2, Ma=0.8,
                  Re=7.0, wall_u=(0.0, 0.4), wall_T=(np.full(nx, 1.1), np.full(nx, 0.9)))
    box = O3.Box(d=(dx, dy, dz), bc=(O3.PERIODIC if periodic else O3.INLET_OUTLET, O3.WALLS,
                                     O3.PERIODIC),
                 wall_vel=(((0, 0, 0), (0, 0, 0)), ((0, 0, 0), (0.4, 0, 0)), ((0, 0, 0), (0, 0, 0))),
                 wall_T=((1, 1), (1.1, 0.9), (1, 1)), Ma=0.8, Re=7.0, g=(0.3, -0.2, 0.0))
    u = 1.0 + 0.1 * rng.normal(size=(ny, nx + 1))
    v = 0.1 * rng.normal(size=(ny + 1, nx))
    pr = 1.0 + 0.05 * rng.uniform(-1, 1, (ny, nx))
    T = 1.0 + 0.05 * rng.uniform(-1, 1, (ny, nx))
    if periodic:
        u[:, -1] = u[:, 0]
    return p, box, (u, v, pr, T), nz, dz[0]


def _set_both(o2, o3, st, nz):
    u, v, pr, T = st
    ext = lambda a: np.repeat(a[None], nz, 0)
    o2.set_fields(u, v, pr, T)
    o3.set_fields(ext(u), ext(v), np.zeros((nz + 1,) + pr.shape), ext(pr), ext(T))


@pytest.mark.parametrize("scheme", list(O3.SCHEMES.values()))
@pytest.mark.parametrize("periodic", [False, True])
def test_z_invariant_equations_are_the_2d_equations(scheme, periodic):
    # every coefficient carries the z width of its volume once, so the 3-D
    # residual is dz times the 2-D one; the w-equation of a flow with w = 0
    # and no z dependence is satisfied exactly.  (The pressure equation's
    # coefficients d = A area / a0 also hold the z conductances of a0, so it
    # is compared through the converged steps below.)
    p, box, st, nz, dz = _pair(periodic, 7)
    o2, o3 = O.Oracle(p), O3.Oracle3(box)
    _set_both(o2, o3, st, nz)
    rT, ru, rv, _ = o2.eq_residuals(0.013, scheme)
    r3 = o3.eq_residuals(0.013, scheme)
    for a, b, name in ((r3[0], ru, "u"), (r3[1], rv, "v"), (r3[4], rT, "T")):
        scale = np.abs(b).max()
        assert scale > 1e-4, name
        assert np.abs(a / dz - b[None]).max() <= 1e-13 * scale, name
    assert np.all(r3[2] == 0.0)


@pytest.mark.parametrize("scheme", list(O3.SCHEMES.values()))
@pytest.mark.parametrize("periodic", [False, True])
def test_z_invariant_steps_are_the_2d_steps(scheme, periodic):
    # with loop 2 run to convergence both oracles reach the solution of the
    # same discrete system in every step
    p, box, st, nz, dz = _pair(periodic, 11)
    o2, o3 = O.Oracle(p), O3.Oracle3(box)
    _set_both(o2, o3, st, nz)
    for _ in range(2):
        o2.step(0.002, 60, scheme)
        o3.step(0.002, 60, scheme)
    assert o2.residuals()[:4].max() < 1e-14
    f2, f3 = o2.fields(), o3.fields()
    for k, j in ((0, 0), (1, 1), (3, 2), (4, 3)):
        assert np.abs(f3[k] - f2[j][None]).max() <= 5e-15 * max(1.0, np.abs(f2[j]).max()), k
    assert np.all(f3[2] == 0.0)
    assert np.abs(f2[0] - st[0]).max() > 1e-4  # the flow did change


# ---------------------------------------------------------------------------
# exchanging two axes commutes with the discrete equations
# ---------------------------------------------------------------------------
def _swap_box(box, e1, e2):
    sig = [0, 1, 2]
    sig[e1], sig[e2] = e2, e1

    def comp(vec):
        return tuple(vec[sig[k]] for k in range(3))

    return O3.Box(d=comp(box.d), bc=comp(box.bc), wall_type=comp(box.wall_type),
                  wall_vel=tuple(tuple(comp(box.wall_vel[sig[e]][s]) for s in range(2))
                                 for e in range(3)),
                  wall_T=comp(box.wall_T), Ma=box.Ma, Re=box.Re, Pr=box.Pr, gamma=box.gamma,
                  u_in=box.u_in, T_in=box.T_in, p_in=box.p_in, g=comp(box.g))


def _swap_fields(f, e1, e2):
    # numpy axis of direction e is 2 - e; component e becomes component sig(e)
    sig = [0, 1, 2]
    sig[e1], sig[e2] = e2, e1
    sw = [np.swapaxes(a, 2 - e1, 2 - e2) for a in f]
    return [sw[sig[0]], sw[sig[1]], sw[sig[2]], sw[3], sw[4]]


@pytest.mark.parametrize("scheme", list(O3.SCHEMES.values()))
@pytest.mark.parametrize("case", ["yz_walls", "xy_periodic", "xz_periodic"])
def test_axis_exchange_commutes_with_the_equations(scheme, case):
    rng = np.random.default_rng(5)
    d = (rng.uniform(0.05, 0.2, 7), rng.uniform(0.05, 0.2, 6), rng.uniform(0.05, 0.2, 5))
    if case == "yz_walls":
        e1, e2 = 1, 2
        box = O3.Box(d=d, bc=(O3.PERIODIC, O3.WALLS, O3.WALLS),
                     wall_type=((O3.NOSLIP, O3.NOSLIP), (O3.NOSLIP, O3.SLIP), (O3.SLIP, O3.NOSLIP)),
                     wall_vel=(((0, 0, 0), (0, 0, 0)), ((0.3, 0, -0.2), (0, 0, 0)),
                               ((0, 0, 0), (-0.1, 0.25, 0))),
                     wall_T=((1, 1), (1.2, 1.0), (1.0, 0.85)), Ma=0.9, Re=6.0, g=(0.2, -0.3, 0.4))
    else:
        e1, e2 = (0, 1) if case == "xy_periodic" else (0, 2)
        box = O3.Box(d=d, bc=(O3.PERIODIC,) * 3, Ma=0.9, Re=6.0, g=(0.2, -0.3, 0.4))
    f = [0.2 * rng.normal(size=s) for s in box.shapes()]
    f[0] += 0.5
    f[3] = 1.0 + 0.1 * rng.uniform(-1, 1, f[3].shape)
    f[4] = 1.0 + 0.1 * rng.uniform(-1, 1, f[4].shape)
    oa = O3.Oracle3(box)
    oa.set_fields(*f)
    fa = oa.fields()  # boundary values imposed
    ra = oa.eq_residuals(0.011, scheme)
    boxb = _swap_box(box, e1, e2)
    ob = O3.Oracle3(boxb)
    ob.set_fields(*_swap_fields(fa, e1, e2))
    rb = ob.eq_residuals(0.011, scheme)
    for k, (x, y) in enumerate(zip(_swap_fields(ra, e1, e2), rb)):
        scale = np.abs(x).max()
        assert scale > 1e-4, k
        assert np.abs(x - y).max() <= 1e-13 * scale, k


# ---------------------------------------------------------------------------
# compressible Couette flow, wall moving in an oblique direction
# ---------------------------------------------------------------------------
_CO = dict(Ma=1.0, Re=5.0, Pr=0.7, gamma=1.4)
_TB, _TT, _U = 1.0, 1.2, (0.6, 0.8)


def _couette3(N, wall_dir):
    # walls normal to wall_dir, the moving wall's velocity (0.6, 0.8) in the
    # other two directions, |U| = 1: the closed form of the 1-D problem with
    # U = 1 gives u_t / U_t for both tangential components
    n = 4
    tang = [e for e in range(3) if e != wall_dir]
    d = [np.full(n, 0.5 / n)] * 3
    d[wall_dir] = np.full(N, 1.0 / N)
    bc = [O3.PERIODIC] * 3
    bc[wall_dir] = O3.WALLS
    top = [0.0, 0.0, 0.0]
    top[tang[0]], top[tang[1]] = _U
    wv = [((0, 0, 0), (0, 0, 0))] * 3
    wv[wall_dir] = ((0, 0, 0), tuple(top))
    wT = [(1, 1)] * 3
    wT[wall_dir] = (_TB, _TT)
    box = O3.Box(d=tuple(d), bc=tuple(bc), wall_vel=tuple(wv), wall_T=tuple(wT), **_CO)
    y = (np.arange(N) + 0.5) / N
    shape = [1, 1, 1]
    shape[2 - wall_dir] = N
    prof = lambda a: a.reshape(shape)
    f = [np.zeros(s) for s in box.shapes()]
    for k, e in enumerate(tang):
        f[e][:] = prof(_U[k] * y)
    f[3][:] = 1.0
    f[4][:] = prof(_TB + (_TT - _TB) * y)
    o = O3.Oracle3(box)
    o.set_fields(*f)
    for s in range(4000):
        o.step(0.02, 20, O3.IMPLICIT | O3.UPWIND)
        if s > 5 and o.residuals()[:5].max() < 1e-13:
            break
    else:
        raise AssertionError("no steady state")
    fl = o.fields()
    line = lambda a: np.moveaxis(a, 2 - wall_dir, 0)[:N, 0, 0]
    K = (_CO["gamma"] - 1) * _CO["Ma"] ** 2 * _CO["Pr"]
    ex = _couette_exact(y, 1.0, _TB, _TT, K)
    s0, s1 = line(fl[tang[0]]) / _U[0], line(fl[tang[1]]) / _U[1]
    # the two tangential components share one profile; the normal one is 0
    assert np.abs(s0 - s1).max() <= 1e-12
    assert np.abs(fl[wall_dir]).max() < 1e-6
    for e in tang:  # no dependence on the periodic directions
        assert np.abs(fl[e] - line(fl[e]).reshape(shape)).max() <= 1e-12 * (1 + np.abs(fl[e]).max())
    return np.abs(s0 - ex[:, 0]).max(), np.abs(line(fl[4]) - ex[:, 1]).max()


def test_couette_between_y_walls_converges_at_second_order():
    e = np.array([_couette3(N, 1) for N in (8, 16, 32)])
    order_u, order_T = np.log2(e[:-1, 0] / e[1:, 0]), np.log2(e[:-1, 1] / e[1:, 1])
    assert np.all((order_T > 1.9) & (order_T < 2.1)), order_T
    assert order_u[-1] > 1.7, order_u
    assert e[-1, 0] < 2e-7 and e[-1, 1] < 5e-5, e[-1]


def test_couette_between_z_walls():
    # the same flow turned so that the walls are normal to z (the z-wall
    # conductances, wall velocities and wall temperatures)
    eu, eT = _couette3(16, 2)
    assert eu < 4e-7 and eT < 1.6e-4, (eu, eT)


# ---------------------------------------------------------------------------
# mass in a closed box
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", list(O3.SCHEMES.values()))
def test_converged_passes_conserve_mass_in_a_closed_box(scheme):
    rng = np.random.default_rng(9)
    box = O3.Box(d=(rng.uniform(0.1, 0.2, 6), rng.uniform(0.1, 0.2, 5), rng.uniform(0.1, 0.2, 5)),
                 bc=(O3.PERIODIC, O3.WALLS, O3.WALLS),
                 wall_vel=(((0, 0, 0), (0, 0, 0)), ((0, 0, 0), (0.3, 0, 0.1)), ((0, 0, 0), (0, 0.2, 0))),
                 wall_T=((1, 1), (1.1, 0.9), (1.0, 1.05)), Ma=0.5, Re=10.0, g=(0.0, -0.5, 0.2))
    f = [0.1 * rng.normal(size=s) for s in box.shapes()]
    f[3] = 1.0 + 0.05 * rng.uniform(-1, 1, f[3].shape)
    f[4] = 1.0 + 0.05 * rng.uniform(-1, 1, f[4].shape)
    o = O3.Oracle3(box)
    o.set_fields(*f)
    m0 = o.mass()
    for _ in range(3):
        o.step(0.005, 80, scheme)
        r = o.residuals()
        assert r[:5].max() < 1e-13, r
        assert abs(r[6]) <= 1e-12 * m0, r
    assert abs(o.mass() - m0) <= 1e-12 * m0


def test_create_refuses_grids_below_four_cells():
    with pytest.raises(ValueError):
        O3.Oracle3(O3.Box(d=(np.ones(4), np.ones(3), np.ones(4))))
