"""Pins of the three-dimensional oracle's discrete operators against the
continuous equations (manufactured solutions; CPU only).

As the two-dimensional manufactured test does for ora.c: smooth analytic
fields u, v, w, p, T are sampled on the staggered grid and frozen as both the
previous time level and the old iterate, and the oracle evaluates every
discrete equation in coefficient form (ora3_eq_residuals).  The unsteady
terms cancel, so the residual of a control volume is the discrete
counterpart of the steady operator integrated over that volume:
  q_a (a = x, y, z):  div(rho u q_a) + A d_a p - B sum_b d_b tau_ab
  T:                  div(rho u T) - C1 div(Gamma grad T) - C2 Gamma Phi
                      - C3 p div(u)
  p:                  dt div(rho u)                         (dt -> 0)
with tau_ab = Gamma (d_a q_b + d_b q_a - 2/3 delta_ab div u) and
Phi = 2 sum_a (d_a q_a)^2 + sum_{a<b} (d_a q_b + d_b q_a)^2 - 2/3 (div u)^2:
the 2-D equations of Sec. 2 and Sec. 3.2 (eqs pl2-pl6, pl14-pl16,
pl28-pl33) read for three directions, with the constants of the hard-sphere
nondimensionalisation (eqs pl35-pl37): A = 1/(gamma Ma^2), B = 1/Re,
C1 = gamma/(Re Pr), C2 = gamma (gamma-1) Ma^2/Re, C3 = -(gamma-1),
Gamma = sqrt(T).

The residuals are linear in those constants, so evaluating them at two
values of Re, of Ma, of Pr and of gamma separates the viscous stress, the
pressure gradient, the conduction, the dissipation, the pressure work and
the convection.  Over the volumes of a central block each part is compared
with the integral of its continuous operator (automatic differentiation in
FP64, 3x3x3 Gauss rule) and must converge under refinement at its
truncation order, on uniform and smoothly stretched grids: second for the
viscous stresses of all three components (the 4/3 normal factors, the
cross-diffusion of every tangential direction, Gamma on the cell edges), the
conduction with harmonic means, the dissipation with all six strain terms,
the pressure work and the pressure gradient; convection and continuity
second with TVD and first with upwind (the fields are monotone in every
direction over the block and its stencils, so the van Leer limiter never
clips).  This pins every term in z directly, beside the symmetry and 2-D
reduction pins of the 3-D oracle.
"""
from __future__ import annotations

import functools
import math

import numpy as np
import pytest
import torch

from oracle import oracle3 as O3

GL = np.array([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)])
GW = np.array([5 / 9, 8 / 9, 5 / 9])
BASE = dict(Ma=2.0, Re=20.0, Pr=0.7, gamma=1.4)
BLOCK = (0.34, 0.66)     # the volumes checked: centres in this cube
SIGNS = (1, -1, 1)       # stretching direction per axis


@pytest.fixture(scope="module", autouse=True)
def _threads():
    # every evaluation is one pass over the grid: four threads, restored for
    # the modules that follow (the OpenMP setting is per process)
    from oracle import oracle as O
    prev = O.max_threads()
    O3.set_threads(4)
    yield
    O3.set_threads(prev)


def fields(x, y, z):
    """Smooth fields whose first derivatives (and those of rho = p/T) keep
    one sign over [0.15, 0.85]^3 (checked in test_fields_are_monotone)."""
    u = 0.7 + 0.25 * x + 0.1 * torch.sin(0.8 * y + 0.3 * x + 0.2 * z) + 0.05 * x * x + 0.04 * z
    v = 0.1 + 0.15 * torch.sin(0.9 * x + 0.5) * (0.5 + y) + 0.05 * z
    w = -0.05 + 0.1 * x + 0.08 * y + 0.12 * torch.sin(0.7 * z + 0.4)
    T = 1.0 + 0.2 * x - 0.15 * y + 0.04 * z + 0.05 * x * y + 0.05 * x * x - 0.01 * y * z
    p = (1.2 - 0.2 * x + 0.1 * y * y - 0.03 * x * y - 0.02 * x ** 3 + 0.05 * x * y * y
         + 0.04 * x * x * y + 0.15 * z + 0.02 * x * z + 0.04 * z * z + 0.03 * y * z * z
         + 0.05 * x * x * z)
    return u, v, w, p, T


def consts(Ma, Re, Pr, gamma):
    return (1.0 / (gamma * Ma * Ma), 1.0 / Re, gamma / (Re * Pr),
            gamma * (gamma - 1.0) * Ma * Ma / Re, -(gamma - 1.0))


def operators(x, y, z):
    """The continuous operators at the points (x, y, z) (flat tensors)."""
    X = [t.clone().requires_grad_(True) for t in (x, y, z)]
    u, v, w, p, T = fields(*X)
    q = (u, v, w)

    def g(f):
        return torch.autograd.grad(f.sum(), X, create_graph=True)

    dq = [g(c) for c in q]                  # dq[a][b] = d_b q_a
    gT, gp = g(T), g(p)
    div = dq[0][0] + dq[1][1] + dq[2][2]
    G, rho = torch.sqrt(T), p / T
    out = {}
    for a in range(3):
        visc = 0.0
        conv = 0.0
        for b in range(3):
            tau = G * (dq[a][b] + dq[b][a] - (2.0 / 3.0 * div if a == b else 0.0))
            visc = visc + g(tau)[b]
            conv = conv + g(rho * q[b] * q[a])[b]
        out[f"visc{a}"], out[f"conv{a}"], out[f"pg{a}"] = visc, conv, gp[a]
    out["cond"] = sum(g(G * gT[b])[b] for b in range(3))
    phi = 2.0 * (dq[0][0] ** 2 + dq[1][1] ** 2 + dq[2][2] ** 2) - 2.0 / 3.0 * div ** 2
    for a in range(3):
        for b in range(a + 1, 3):
            phi = phi + (dq[a][b] + dq[b][a]) ** 2
    out["diss"] = G * phi
    out["pw"] = p * div
    out["convT"] = sum(g(rho * q[b] * T)[b] for b in range(3))
    out["cont"] = sum(g(rho * q[b])[b] for b in range(3))
    return {k: t.detach().numpy() for k, t in out.items()}


def box_integrals(lo, hi):
    """Integrals of the operators over the boxes [lo, hi] (arrays (n, 3))."""
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    n = len(lo)
    pts = []
    for e, shp in enumerate(((3, 1, 1), (1, 3, 1), (1, 1, 3))):
        pe = mid[:, e, None, None, None] + half[:, e, None, None, None] * GL.reshape(shp)[None]
        pts.append(np.broadcast_to(pe, (n, 3, 3, 3)).reshape(-1))
    nt = torch.get_num_threads()
    torch.set_num_threads(1)
    torch.set_flush_denormal(True)
    try:
        ops = operators(*[torch.tensor(a.copy(), dtype=torch.float64) for a in pts])
    finally:
        torch.set_num_threads(nt)
        torch.set_flush_denormal(False)
    wgt = (GW[:, None, None] * GW[None, :, None] * GW[None, None, :]).reshape(-1)
    jac = half.prod(axis=1)
    return {k: (a.reshape(n, 27) * wgt).sum(axis=1) * jac for k, a in ops.items()}


def stretch(N, a, sign):
    e = np.arange(N + 1) / N
    return e + sign * a * np.sin(2 * math.pi * e) / (2 * math.pi)


@functools.lru_cache(maxsize=None)
def grid(N, a):
    f = [stretch(N, a, s) for s in SIGNS]
    c = [0.5 * (x[1:] + x[:-1]) for x in f]
    return f, c


def volumes(N, a):
    """Index sets and bounds of the checked volumes: per unknown kind (u, v,
    w faces; cells) the (k, j, i) indices in its array and the box bounds."""
    f, c = grid(N, a)
    inb = lambda t: (t > BLOCK[0]) & (t < BLOCK[1])
    out = {}
    for kind in range(4):               # 0, 1, 2: faces normal to x, y, z; 3: cells
        axes = []
        for e in range(3):
            if e == kind:               # face index i: volume from centre i-1 to centre i
                idx = np.arange(1, N)
                lo, hi, pos = c[e][idx - 1], c[e][idx], f[e][idx]
            else:
                idx = np.arange(N)
                lo, hi, pos = f[e][idx], f[e][idx + 1], c[e][idx]
            m = inb(pos)
            axes.append((idx[m], lo[m], hi[m]))
        (ix, xl, xh), (iy, yl, yh), (iz, zl, zh) = axes
        K, J, I = np.meshgrid(iz, iy, ix, indexing="ij")
        LO = np.stack(np.meshgrid(zl, yl, xl, indexing="ij")[::-1], -1).reshape(-1, 3)
        HI = np.stack(np.meshgrid(zh, yh, xh, indexing="ij")[::-1], -1).reshape(-1, 3)
        out[kind] = ((K.reshape(-1), J.reshape(-1), I.reshape(-1)), LO, HI)
    return out


@functools.lru_cache(maxsize=None)
def exact(N, a):
    return {kind: box_integrals(lo, hi) for kind, (_, lo, hi) in volumes(N, a).items()}


def sample(N, a):
    """u at (x^f_i, y_j, z_k), v at (x_i, y^f_j, z_k), w at (x_i, y_j, z^f_k),
    p and T at the cell centres, in the oracle's (z, y, x) layouts."""
    f, c = grid(N, a)
    tt = lambda g: torch.tensor(g, dtype=torch.float64)

    def at(xs, ys, zs, which):
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        return fields(tt(X), tt(Y), tt(Z))[which].numpy()
    return [at(f[0], c[1], c[2], 0), at(c[0], f[1], c[2], 1), at(c[0], c[1], f[2], 2),
            at(c[0], c[1], c[2], 3), at(c[0], c[1], c[2], 4)]


def parts(N, a, scheme):
    f, _ = grid(N, a)
    q = sample(N, a)

    def resid(dt=1.0, **kw):
        prm = {**BASE, **kw}
        box = O3.Box(d=tuple(np.diff(x) for x in f),
                     bc=(O3.INLET_OUTLET, O3.WALLS, O3.WALLS), u_in=0.9, T_in=1.0, p_in=1.1,
                     **prm)
        o = O3.Oracle3(box)
        o.set_fields(*q)
        return o.eq_residuals(dt, scheme)

    r0, rRe, rMa, rPr, rg = (resid(), resid(Re=40.0), resid(Ma=1.5), resid(Pr=1.4),
                             resid(gamma=1.6))
    rp = resid(dt=1e-7)[3]
    P0, PRe, PMa, PPr, Pg = (consts(**BASE), consts(**{**BASE, "Re": 40.0}),
                             consts(**{**BASE, "Ma": 1.5}), consts(**{**BASE, "Pr": 1.4}),
                             consts(**{**BASE, "gamma": 1.6}))
    out = {}
    for e in range(3):
        out[f"visc{e}"] = (r0[e] - rRe[e]) / (P0[1] - PRe[1])
        out[f"pg{e}"] = (r0[e] - rMa[e]) / (P0[0] - PMa[0])
        out[f"conv{e}"] = r0[e] - P0[0] * out[f"pg{e}"] - P0[1] * out[f"visc{e}"]
    rT = r0[4]
    out["cond"] = (rT - rPr[4]) / (P0[2] - PPr[2])
    out["diss"] = (rT - rMa[4]) / (P0[3] - PMa[3])
    out["pw"] = (((rT - rg[4]) - (P0[2] - Pg[2]) * out["cond"] - (P0[3] - Pg[3]) * out["diss"])
                 / (P0[4] - Pg[4]))
    out["convT"] = rT - P0[2] * out["cond"] - P0[3] * out["diss"] - P0[4] * out["pw"]
    out["cont"] = rp / 1e-7
    return out


# sign of each continuous part in the residual
SIGN = {**{f"visc{e}": -1 for e in range(3)}, **{f"pg{e}": 1 for e in range(3)},
        **{f"conv{e}": 1 for e in range(3)}, "cond": -1, "diss": -1, "pw": -1, "convT": 1,
        "cont": 1}
KIND = {**{f"{p}{e}": e for p in ("visc", "pg", "conv") for e in range(3)},
        "cond": 3, "diss": 3, "pw": 3, "convT": 3, "cont": 3}


def errors(N, a, scheme):
    """Max error of every discrete part over the block's volumes relative to
    the largest exact value."""
    d = parts(N, a, scheme)
    vol, ex = volumes(N, a), exact(N, a)
    err = {}
    for k, kind in KIND.items():
        idx = vol[kind][0]
        ref = SIGN[k] * ex[kind][k]
        err[k] = float(np.abs(d[k][idx] - ref).max() / np.abs(ref).max())
    return err


SECOND = tuple(f"visc{e}" for e in range(3)) + tuple(f"pg{e}" for e in range(3)) + (
    "cond", "diss", "pw")


def test_fields_are_monotone():
    g = torch.linspace(0.15, 0.85, 29, dtype=torch.float64)
    X = [t.reshape(-1).clone().requires_grad_(True) for t in torch.meshgrid(g, g, g, indexing="ij")]
    u, v, w, p, T = fields(*X)
    for f in (u, v, w, p, T, p / T):
        for d in torch.autograd.grad(f.sum(), X, retain_graph=True):
            assert bool((d > 0).all()) or bool((d < 0).all())


@pytest.mark.parametrize("a", [0.0, 0.5], ids=["uniform", "stretched"])
@pytest.mark.parametrize("name,scheme", list(O3.SCHEMES.items()))
def test_3d_operators_converge_to_the_equations(a, name, scheme):
    Ns = (12, 24, 48)
    errs = [errors(N, a, scheme) for N in Ns]
    conv_order = 2.0 if scheme & O3.TVD else 1.0
    for k in errs[0]:
        e = [x[k] for x in errs]
        order = math.log2(e[1] / e[2])     # the finer pair (12 cells per unit are pre-asymptotic)
        print(f"{name} a={a} {k:6s} " + " ".join(f"{x:.2e}" for x in e) + f"  order {order:.2f}")
        if k in SECOND or conv_order == 2.0:
            assert order >= 1.7 and e[2] < 1e-2, (k, e, order)
        else:
            assert 0.7 <= order <= 1.3 and e[2] < 0.1, (k, e, order)
