"""Pins of the oracle's tangent-linear model (ora.c compiled on the dual
numbers of oracle/tlm.h; test infrastructure of the adjoint tests).

- Its values are the oracle's, bitwise: the dual arithmetic carries the
  plain FP64 value through every operation and branch.
- Its tangents are the derivatives of the oracle's loss: on a small channel
  with an obstacle, heated walls and a seeded parabolic inlet (12 explicit
  steps of 4 passes: explicit upwind and TVD, implicit upwind; implicit TVD
  is discontinuous at limiter ties and has no derivative there), the
  directional derivatives of
  the time-averaged drag along 16 seeded directions in the inlet profile,
  the wall temperatures and the initial state agree with central
  differences of the oracle's loss (h = 1e-7; measured 4e-9 .. 3e-8).
"""
from __future__ import annotations

import copy

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W


def small_case():
    nx, ny = 24, 10
    x = (np.arange(nx) + 0.5) / nx
    return W.Problem(nx=nx, ny=ny, lx=2.4, ly=1.0, obstacles=[(3, 3, 5, 6)], Re=20.0,
                     u_in=W.parabolic_inlet(ny, 7),
                     wall_T=(1.0 + 0.05 * np.sin(2 * np.pi * x), 1.0 - 0.03 * np.cos(np.pi * x)))


@pytest.mark.parametrize("name,scheme", [("explicit_upwind", W.EXPLICIT | W.UPWIND),
                                         ("explicit_tvd", W.EXPLICIT | W.TVD),
                                         ("implicit_upwind", W.IMPLICIT | W.UPWIND)])
def test_tangent_linear_model_matches_central_differences(oracle_lib, name, scheme):
    p = small_case()
    f0 = W.initial_fields(p, 11)
    dt, steps, inner = p.cfl_dt(), 12, 4
    K = oracle_lib.tlm_lib().tlm_k()
    rng = np.random.default_rng(5)
    du = rng.standard_normal((K, p.ny))
    dw0, dw1 = rng.standard_normal((K, p.nx)), rng.standard_normal((K, p.nx))
    df = [rng.standard_normal((K,) + a.shape) for a in f0]
    t = oracle_lib.Tangent(p, du, (dw0, dw1))
    t.set_fields(f0, df)
    o = oracle_lib.Oracle(p)
    o.set_fields(*f0)
    acc = np.zeros(K)
    for _ in range(steps):
        t.step(dt, inner, scheme)
        o.step(dt, inner, scheme)
        vals, tans = t.fields()
        for a, b in zip(vals, o.fields()):
            assert np.array_equal(a, b)
        acc += oracle_lib.drag_tangent(p, vals, tans)[1]
    tlm = acc / steps

    def loss(eps, k):
        q = copy.copy(p)
        q.u_in = p.u_in + eps * du[k]
        q.wall_T = (p.wall_T[0] + eps * dw0[k], p.wall_T[1] + eps * dw1[k])
        r = oracle_lib.Oracle(q)
        r.set_fields(*[a + eps * d[k] for a, d in zip(f0, df)])
        L = 0.0
        for _ in range(steps):
            r.step(dt, inner, scheme)
            L += oracle_lib.drag(q, r.fields())
        return L / steps

    h = 1e-7
    rels = []
    for k in range(K):
        fd = (loss(h, k) - loss(-h, k)) / (2 * h)
        rels.append(abs(tlm[k] - fd) / abs(fd))
        print(f"{name} direction {k}: tangent-linear {tlm[k]:.12e} fd {fd:.12e} rel {rels[-1]:.1e}")
    # the difference quotient carries O(h^2) truncation and O(eps/h)
    # round-off: ~1e-8, up to ~1e-6 where a direction curves strongly
    assert np.median(rels) <= 1e-7 and max(rels) <= 1e-5, rels
