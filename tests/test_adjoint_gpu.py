"""Adjoint of the explicit-scheme step (GPU, through the C ABI and the
torch.autograd.Function of paper_1802_04243_amd.adjoint).

Loss: the drag on the obstacle averaged over the steps; parameters: the
inlet profile u_in[ny] and the two wall temperatures wall_T[0][nx],
wall_T[1][nx].  Checks, at relative error 1e-5:
- against an FP64 CPU reference gradient: central differences (h = 1e-6) of
  the oracle's loss in every parameter, on a small channel with one
  obstacle, heated walls and a seeded parabolic inlet (upwind and TVD);
- on the 1024x256 channel (one centred square), a dot-product test against
  the oracle's tangent-linear model (the oracle compiled on dual numbers,
  every branch taken on the value: the derivative of the same piecewise
  smooth step, with no difference quotient across upwind or limiter
  kinks) along 16 seeded directions, 6 in the inlet profile, 5 in the wall
  temperatures and 5 in the initial state around the square: one step of 10
  passes (both spatial schemes) and the configured 100 steps x 10 passes
  with checkpoints every 10 steps (TVD).  In 100 steps the drag feels the
  inlet 486 cells upstream and the walls 96 cells away only through many
  Jacobi passes (derivatives ~1e-224 and ~1e-15), but both sides carry
  them exactly, so each direction is held to 1e-5 relative;
- the same dot-product test for one step of a 2048x512 channel, a grid of
  more than 4096 tiles of the reverse kernels.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
H = 1e-6


def small_case():
    # the obstacle three cells from the inlet and the walls: within 12 steps
    # the inlet and wall values reach the drag at FP64 resolution
    nx, ny = 24, 10
    x = (np.arange(nx) + 0.5) / nx
    return W.Problem(nx=nx, ny=ny, lx=2.4, ly=1.0, obstacles=[(3, 3, 5, 6)], Re=20.0,
                     u_in=W.parabolic_inlet(ny, 7),
                     wall_T=(1.0 + 0.05 * np.sin(2 * np.pi * x), 1.0 - 0.03 * np.cos(np.pi * x)))


def with_params(p, u_in, Tw0, Tw1):
    import copy
    q = copy.copy(p)
    q.u_in, q.wall_T = np.array(u_in), (np.array(Tw0), np.array(Tw1))
    return q


def oracle_loss(oracle_lib, p, f0, dt, steps, inner, scheme):
    o = oracle_lib.Oracle(p)
    o.set_fields(*f0)
    acc = 0.0
    for _ in range(steps):
        o.step(dt, inner, scheme)
        acc += oracle_lib.drag(p, o.fields())
    return acc / steps


def adjoint_gradient(p, f0, dt, steps, inner, scheme, every, fields=False):
    import torch
    from paper_1802_04243_amd import adjoint
    wb, wt = p.walls()
    u = torch.tensor(p.inlet()[0], dtype=torch.float64, requires_grad=True)
    w0 = torch.tensor(wb, dtype=torch.float64, requires_grad=True)
    w1 = torch.tensor(wt, dtype=torch.float64, requires_grad=True)
    ft = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in f0]
    L = adjoint.drag_loss(p, u, w0, w1, ft, dt, steps, inner, scheme, every)
    L.backward()
    out = (float(L.detach()), u.grad.numpy().copy(), w0.grad.numpy().copy(), w1.grad.numpy().copy())
    if fields:
        out = out + (tuple(a.grad.numpy().copy() for a in ft),)
    return out


@pytest.mark.parametrize("name,scheme", [("explicit_upwind", W.EXPLICIT | W.UPWIND),
                                         ("explicit_tvd", W.EXPLICIT | W.TVD)])
def test_adjoint_vs_oracle_gradient(sts_mod, oracle_lib, name, scheme):
    p = small_case()
    f0 = W.initial_fields(p, 11)
    dt, steps, inner = p.cfl_dt(), 12, 4
    print(f"case adjoint 40x12 {name} {steps}x{inner}", flush=True)
    L, gu, g0, g1 = adjoint_gradient(p, f0, dt, steps, inner, scheme, every=5)
    Lo = oracle_loss(oracle_lib, p, f0, dt, steps, inner, scheme)
    assert abs(L - Lo) <= 1e-12 * max(1.0, abs(Lo)), (L, Lo)
    params = [p.u_in.copy(), p.wall_T[0].copy(), p.wall_T[1].copy()]
    for which, g in enumerate((gu, g0, g1)):
        fd = np.zeros_like(params[which])
        for k in range(fd.size):
            pp = [a.copy() for a in params]
            pm = [a.copy() for a in params]
            pp[which][k] += H
            pm[which][k] -= H
            fd[k] = (oracle_loss(oracle_lib, with_params(p, *pp), f0, dt, steps, inner, scheme) -
                     oracle_loss(oracle_lib, with_params(p, *pm), f0, dt, steps, inner, scheme)) / (2 * H)
        err = np.abs(g - fd).max() / np.abs(fd).max()
        print(f"adjoint-vs-oracle-fd {name} {('u_in', 'wall_T0', 'wall_T1')[which]}: "
              f"max|grad| {np.abs(fd).max():.3e}, normwise rel err {err:.2e}", flush=True)
        assert np.isfinite(g).all()
        assert err <= TOL, (which, err)


def tlm_directions_1024x256(oracle_lib, steps, scheme, every):
    from paper_1802_04243_amd import workloads as W_
    p, run = W_.workload("adjoint_1024x256")
    return tlm_directions(oracle_lib, p, run, steps, scheme, every)


def tlm_directions(oracle_lib, p, run, steps, scheme, every):
    """Dot-product test on a channel with one square: the adjoint's directional
    derivatives <gradient, delta> against the oracle's tangent-linear model
    (ora.c compiled on dual numbers: the exact derivative of the branch the
    forward takes) along K seeded directions: 6 in the inlet profile, 5 in
    both wall temperatures, the rest in the initial state around the
    square.  Returns (adjoint, tangent-linear) per direction."""
    f0 = W.initial_fields(p, run["seed"])
    dt, inner = run["dt"], run["inner"]
    K = oracle_lib.tlm_lib().tlm_k()
    print(f"case adjoint dot-product {p.nx}x{p.ny} {steps}x{inner} every {every} scheme {scheme} "
          f"({K} directions)", flush=True)
    L, gu, g0, g1, gf = adjoint_gradient(p, f0, dt, steps, inner, scheme, every, fields=True)
    print(f"L {L:.12e}; max|dL/du_in| {np.abs(gu).max():.2e}, max|dL/dwall_T| "
          f"{max(np.abs(g0).max(), np.abs(g1).max()):.2e}", flush=True)
    rng = np.random.default_rng(2024)
    nx, ny = p.nx, p.ny
    du = np.zeros((K, ny))
    dw0, dw1 = np.zeros((K, nx)), np.zeros((K, nx))
    df = [np.zeros((K,) + a.shape) for a in f0]
    (i0, j0, i1, j1), = p.obstacles
    box = (slice(max(j0 - 16, 1), j1 + 17), slice(i0 - 16, i1 + 17))
    for k in range(K):
        if k < 6:
            du[k] = rng.standard_normal(ny)
        elif k < 11:
            dw0[k] = rng.standard_normal(nx)
            dw1[k] = rng.standard_normal(nx)
        else:
            for a in df:
                a[k][box] = rng.standard_normal(a[k][box].shape)
    t = oracle_lib.Tangent(p, du, (dw0, dw1))
    t.set_fields(f0, df)
    acc, Lt = np.zeros(K), 0.0
    for n in range(steps):
        t.step(dt, inner, scheme)
        D, dD = oracle_lib.drag_tangent(p, *t.fields())
        acc += dD
        Lt += D
    tlm, Lt = acc / steps, Lt / steps
    assert abs(L - Lt) <= 1e-10 * abs(Lt), (L, Lt)
    ad = np.array([float((gu * du[k]).sum() + (g0 * dw0[k]).sum() + (g1 * dw1[k]).sum() +
                         sum((g * d[k]).sum() for g, d in zip(gf, df))) for k in range(K)])
    for k in range(K):
        kind = "u_in" if k < 6 else ("wall_T" if k < 11 else "state")
        rel = abs(ad[k] - tlm[k]) / abs(tlm[k]) if tlm[k] != 0 else abs(ad[k])
        print(f"direction {k} ({kind}): adjoint {ad[k]:.12e} tangent-linear {tlm[k]:.12e} "
              f"rel {rel:.2e}", flush=True)
    return ad, tlm


def assert_dot_products(ad, tlm):
    # every direction within 1e-5 (a direction whose derivative is exactly
    # zero in the tangent-linear model must be zero in the adjoint too)
    for k, (a, t) in enumerate(zip(ad, tlm)):
        assert np.isfinite(a) and abs(a - t) <= TOL * abs(t), (k, a, t)


@pytest.mark.parametrize("name,scheme", [("explicit_upwind", W.EXPLICIT | W.UPWIND),
                                         ("explicit_tvd", W.EXPLICIT | W.TVD)])
def test_adjoint_dot_product_1024x256_one_step(sts_mod, oracle_lib, name, scheme):
    assert_dot_products(*tlm_directions_1024x256(oracle_lib, 1, scheme, 1))


def test_adjoint_dot_product_1024x256_configured_run(sts_mod, oracle_lib):
    # the configured run: 100 steps x 10 passes, checkpoints every 10 steps
    assert_dot_products(*tlm_directions_1024x256(oracle_lib, 100, W.EXPLICIT | W.TVD, 10))


def test_adjoint_dot_product_2048x512_one_step(sts_mod, oracle_lib):
    # 65 x 65 = 4225 tiles of 32 x 8: the grid size from which the four
    # scatter stages of the reverse pass run as separate launches
    from paper_1802_04243_amd import workloads as W_
    from fractions import Fraction
    p = W_.channel(2048, 512, [Fraction(5, 2)], u_in=W_.parabolic_inlet(512, 4))
    run = dict(inner=10, seed=4, dt=p.cfl_dt())
    assert_dot_products(*tlm_directions(oracle_lib, p, run, 1, W.EXPLICIT | W.TVD, 1))


def test_adjoint_argument_errors(sts_mod):
    p = small_case()
    g = sts_mod.Solver(p)
    with pytest.raises(sts_mod.StsError) as e:
        g.adjoint_step(p.cfl_dt(), 4, W.EXPLICIT)
    assert e.value.code == sts_mod.STS_ESTATE
    g.adjoint_begin(4)
    for bad in (W.IMPLICIT, W.IMPLICIT | W.TVD | W.MIXED):
        with pytest.raises(sts_mod.StsError) as e:
            g.adjoint_step(p.cfl_dt(), 4, bad)
        assert e.value.code == sts_mod.STS_EINVAL
    with pytest.raises(sts_mod.StsError) as e:
        g.adjoint_step(p.cfl_dt(), 5, W.EXPLICIT)
    assert e.value.code == sts_mod.STS_EINVAL
    with pytest.raises(sts_mod.StsError) as e:
        g.state_save(0)
    assert e.value.code == sts_mod.STS_EINVAL
    g.close()
    q = W.Problem(nx=16, ny=8, lx=2.0, periodic=True)
    h = sts_mod.Solver(q)
    with pytest.raises(sts_mod.StsError) as e:
        h.adjoint_begin(4)
    assert e.value.code == sts_mod.STS_EINVAL
    h.close()
