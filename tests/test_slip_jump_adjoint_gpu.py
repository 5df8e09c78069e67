"""Adjoint of the explicit step with velocity-slip / temperature-jump
surfaces (eqs pl38, pl39; GPU, through the C ABI).

The slip / jump conductance Gamma / (d/2 + k/rho) and the slip velocity of
the dissipation term are differentiated in the node's Gamma and rho.
Checked against central differences (h = 1e-6) of the FP64 oracle's loss in
every parameter (inlet profile, both wall temperatures), at normwise
relative error 1e-5, on a 24x10 channel whose walls move and are
slip-jump, with a slip-jump obstacle three cells from the inlet:
- loss: the mean over the steps of a seeded linear functional of the state
  (sts_adjoint_seed at every level), slip-jump walls and obstacle;
- loss: the drag (sts_adjoint_seed_drag) with slip-jump walls around a
  no-slip obstacle;
and in 48 seeded entries of the initial state (its unknowns) against
central differences of the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W

from test_adjoint_gpu import H, TOL, with_params

pytestmark = pytest.mark.gpu

SJ = W.WALL_SLIP_JUMP
SCHEMES = [("explicit_upwind", W.EXPLICIT | W.UPWIND), ("explicit_tvd", W.EXPLICIT | W.TVD)]


def slip_case(obstacle_type=SJ):
    nx, ny = 24, 10
    x = (np.arange(nx) + 0.5) / nx
    return W.Problem(nx=nx, ny=ny, lx=2.4, ly=1.0, obstacles=[(3, 3, 5, 6)], Re=20.0,
                     u_in=W.parabolic_inlet(ny, 7), wall_type=(SJ, SJ), wall_u=(0.2, -0.1),
                     obstacle_type=obstacle_type, kn=0.02,
                     wall_T=(1.0 + 0.05 * np.sin(2 * np.pi * x), 1.0 - 0.03 * np.cos(np.pi * x)))


def weights(p, seed=5):
    rng = np.random.default_rng(seed)
    shapes = ((p.ny, p.nx + 1), (p.ny + 1, p.nx), (p.ny, p.nx), (p.ny, p.nx))
    return [rng.standard_normal(s) for s in shapes]


def oracle_functional(oracle_lib, p, f0, dt, steps, inner, scheme, w):
    o = oracle_lib.Oracle(p)
    o.set_fields(*f0)
    acc = 0.0
    for _ in range(steps):
        o.step(dt, inner, scheme)
        acc += sum(float((a * b).sum()) for a, b in zip(w, o.fields()))
    return acc / steps


def oracle_drag(oracle_lib, p, f0, dt, steps, inner, scheme):
    o = oracle_lib.Oracle(p)
    o.set_fields(*f0)
    acc = 0.0
    for _ in range(steps):
        o.step(dt, inner, scheme)
        acc += oracle_lib.drag(p, o.fields())
    return acc / steps


def gpu_gradient(sts_mod, p, f0, dt, steps, inner, scheme, w=None):
    """Loss and (dL/du_in, dL/dwall_T0, dL/dwall_T1, dL/d(initial state)):
    forward with every level in a device slot, then the reverse with the
    loss's seed added at each level."""
    g = sts_mod.Solver(p)
    g.set_fields(*f0)
    g.state_slots(steps + 1)
    g.state_save(0)
    L = 0.0
    for n in range(1, steps + 1):
        g.step(dt, inner, scheme)
        g.state_save(n)
        L += (sum(float((a * b).sum()) for a, b in zip(w, g.fields())) if w is not None
              else g.drag()) / steps
    g.adjoint_begin(inner)
    for n in range(steps, 0, -1):
        g.state_load(n)
        if w is not None:
            g.adjoint_seed(*[a / steps for a in w])
        else:
            g.adjoint_seed_drag(1.0 / steps)
        g.state_load(n - 1)
        g.adjoint_step(dt, inner, scheme)
    (gu, g0, g1), lam = g.adjoint_read(with_lambda=True)
    g.close()
    return L, gu, g0, g1, lam


def check_params(p, f0, dt, steps, inner, scheme, grads, loss, label):
    params = [p.u_in.copy(), p.wall_T[0].copy(), p.wall_T[1].copy()]
    for which, g in enumerate(grads):
        fd = np.zeros_like(params[which])
        for k in range(fd.size):
            pp = [a.copy() for a in params]
            pm = [a.copy() for a in params]
            pp[which][k] += H
            pm[which][k] -= H
            fd[k] = (loss(with_params(p, *pp)) - loss(with_params(p, *pm))) / (2 * H)
        err = np.abs(g - fd).max() / np.abs(fd).max()
        print(f"{label} {('u_in', 'wall_T0', 'wall_T1')[which]}: max|grad| {np.abs(fd).max():.3e}, "
              f"normwise rel err {err:.2e}", flush=True)
        assert np.isfinite(g).all()
        assert np.abs(fd).max() > 0
        assert err <= TOL, (label, which, err)


@pytest.mark.parametrize("name,scheme", SCHEMES)
def test_slip_jump_adjoint_linear_functional(sts_mod, oracle_lib, name, scheme):
    p = slip_case()
    f0 = W.initial_fields(p, 11)
    w = weights(p)
    dt, steps, inner = p.cfl_dt(), 12, 4
    print(f"case slip-jump adjoint 24x10 functional {name} {steps}x{inner}", flush=True)
    L, gu, g0, g1, lam = gpu_gradient(sts_mod, p, f0, dt, steps, inner, scheme, w)
    Lo = oracle_functional(oracle_lib, p, f0, dt, steps, inner, scheme, w)
    assert abs(L - Lo) <= 1e-12 * max(1.0, abs(Lo)), (L, Lo)
    check_params(p, f0, dt, steps, inner, scheme, (gu, g0, g1),
                 lambda q: oracle_functional(oracle_lib, q, f0, dt, steps, inner, scheme, w),
                 f"slip-jump functional {name}")
    # initial-state derivatives, entry by entry on a seeded sample of the
    # unknowns.  The boundary-value projection of the initial state copies u
    # at face nx-1 to the outlet face nx, so a move of the former moves both:
    # its derivative is the sum of the two adjoint entries.  The step is
    # piecewise smooth (upwind switches, limiter kinks): a difference
    # quotient that straddles a switch is not a derivative, and two step
    # sizes (1e-7, 1e-8) rarely straddle the same one; the closer of the two
    # is asserted within 1e-5 max(1, |fd|)
    lu = lam[0].copy()
    lu[:, p.nx - 1] += lu[:, p.nx]
    lam = (lu,) + tuple(lam[1:])
    solid = p.solid_mask().astype(bool)
    unknown = [np.zeros(a.shape, bool) for a in f0]
    unknown[0][:, 1:p.nx] = ~(solid[:, :-1] | solid[:, 1:])
    unknown[1][1:p.ny, :] = ~(solid[:-1, :] | solid[1:, :])
    unknown[2][:] = ~solid
    unknown[3][:] = ~solid
    rng = np.random.default_rng(9)
    worst = 0.0
    for fld in range(4):
        cand = np.argwhere(unknown[fld])
        for jj, ii in cand[rng.choice(len(cand), 12, replace=False)]:
            fds = []
            for hh in (1e-7, 1e-8):
                d = [np.zeros_like(a) for a in f0]
                d[fld][jj, ii] = hh
                fp = oracle_functional(oracle_lib, p, [a + x for a, x in zip(f0, d)], dt, steps,
                                       inner, scheme, w)
                fm = oracle_functional(oracle_lib, p, [a - x for a, x in zip(f0, d)], dt, steps,
                                       inner, scheme, w)
                fds.append((fp - fm) / (2 * hh))
            ad = lam[fld][jj, ii]
            err = min(abs(ad - f) for f in fds) / max(1.0, abs(fds[0]))
            worst = max(worst, err)
            assert err <= TOL, ("uvpT"[fld], jj, ii, ad, fds)
    print(f"initial-state entries: worst rel err {worst:.2e}", flush=True)


@pytest.mark.parametrize("name,scheme", SCHEMES)
def test_slip_jump_walls_adjoint_drag(sts_mod, oracle_lib, name, scheme):
    p = slip_case(obstacle_type=W.WALL_NOSLIP_ISOTHERMAL)
    f0 = W.initial_fields(p, 11)
    dt, steps, inner = p.cfl_dt(), 12, 4
    print(f"case slip-jump walls adjoint 24x10 drag {name} {steps}x{inner}", flush=True)
    L, gu, g0, g1, _ = gpu_gradient(sts_mod, p, f0, dt, steps, inner, scheme)
    Lo = oracle_drag(oracle_lib, p, f0, dt, steps, inner, scheme)
    assert abs(L - Lo) <= 1e-12 * max(1.0, abs(Lo)), (L, Lo)
    check_params(p, f0, dt, steps, inner, scheme, (gu, g0, g1),
                 lambda q: oracle_drag(oracle_lib, q, f0, dt, steps, inner, scheme),
                 f"slip-jump walls drag {name}")


def test_adjoint_seed_argument_checks(sts_mod):
    p = slip_case()
    g = sts_mod.Solver(p)
    w = weights(p)
    with pytest.raises(sts_mod.StsError) as e:   # before sts_adjoint_begin
        g.adjoint_seed(*w)
    assert e.value.code == sts_mod.STS_ESTATE
    g.adjoint_begin(4)
    with pytest.raises(sts_mod.StsError) as e:   # the drag of a slip-jump obstacle
        g.adjoint_seed_drag(1.0)
    assert e.value.code == sts_mod.STS_EINVAL
    bad = [a.copy() for a in w]
    bad[2][3, 4] = np.nan
    with pytest.raises(sts_mod.StsError) as e:
        g.adjoint_seed(*bad)
    assert e.value.code == sts_mod.STS_EINVAL
    with pytest.raises(ValueError):
        g.adjoint_seed(w[1])                      # wrong shape for u
    g.adjoint_seed(None, None, w[2], None)
    *_, lam = g.adjoint_read(with_lambda=True)
    assert np.array_equal(lam[2], w[2]) and not lam[0].any() and not lam[3].any()
    g.close()
