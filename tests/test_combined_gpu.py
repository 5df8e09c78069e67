"""Mixed-precision forward with the FP64 adjoint, and the sqrt(N)
checkpoint schedule (GPU, through the C ABI and
paper_1802_04243_amd.adjoint).

With scheme bit MIXED the forward and every recompute of the backward run
the mixed-precision pass; the reverse is the FP64 step's transpose at those
states.  Its gradient is therefore the FP64 gradient evaluated along a
trajectory that differs by FP32 rounding of the coefficients: checked
against the gradient through the FP64 forward (itself checked against
central differences of the FP64 oracle) at a normwise relative difference
of 1e-5, on the small channel and on the 4096x1024 combined grid (Re 50, two
squares) for 25 steps and for the configured 500 steps (every parameter
and initial-state gradient).  The sqrt(N) schedule (every=None) must give the
gradient of the every-step schedule to rounding: the two differ only in the
order of recomputation, and the reverse kernels' atomic sums make the result
reproducible to rounding, not bitwise.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W

from test_adjoint_gpu import adjoint_gradient, small_case

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5


def normdiff(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


@pytest.mark.parametrize("name,scheme", [("explicit_upwind", W.EXPLICIT | W.UPWIND),
                                         ("explicit_tvd", W.EXPLICIT | W.TVD)])
def test_mixed_forward_adjoint_small(sts_mod, name, scheme):
    p = small_case()
    f0 = W.initial_fields(p, 11)
    dt, steps, inner = p.cfl_dt(), 12, 4
    print(f"case mixed-forward adjoint 24x10 {name}", flush=True)
    Lm, *gm, fm = adjoint_gradient(p, f0, dt, steps, inner, scheme | W.MIXED, 5, fields=True)
    Lf, *gf, ff = adjoint_gradient(p, f0, dt, steps, inner, scheme, 5, fields=True)
    assert abs(Lm - Lf) <= 1e-6 * abs(Lf), (Lm, Lf)
    assert Lm != Lf    # the mixed form ran
    for nm, a, b in zip(["u_in", "wall_T0", "wall_T1", "u0", "v0", "p0", "T0"],
                        list(gm) + list(fm), list(gf) + list(ff)):
        d = normdiff(a, b)
        print(f"mixed vs fp64 gradient {name} {nm}: max|g| {np.abs(b).max():.3e}, rel {d:.2e}",
              flush=True)
        assert np.isfinite(a).all()
        assert d <= TOL_MIXED, (nm, d)


def test_sqrt_schedule_matches_every_step(sts_mod):
    p = small_case()
    f0 = W.initial_fields(p, 11)
    dt, steps, inner = p.cfl_dt(), 12, 4
    assert math.ceil(math.sqrt(steps)) == 4
    La, *ga, fa = adjoint_gradient(p, f0, dt, steps, inner, W.EXPLICIT | W.TVD, None, fields=True)
    Lb, *gb, fb = adjoint_gradient(p, f0, dt, steps, inner, W.EXPLICIT | W.TVD, 1, fields=True)
    assert La == Lb    # the forward does not depend on the schedule
    for a, b in zip(list(ga) + list(fa), list(gb) + list(fb)):
        assert normdiff(a, b) <= 1e-12


def test_mixed_forward_adjoint_combined_grid(sts_mod):
    # the combined workload's grid and physics, 25 steps (sqrt schedule: 5)
    p, run = W.workload("combined_4096x1024")
    f0 = W.initial_fields(p, run["seed"])
    steps, inner, scheme = 25, run["inner"], W.EXPLICIT | W.TVD
    print(f"case combined 4096x1024 {steps}x{inner} mixed forward vs fp64", flush=True)
    Lm, *gm, fm = adjoint_gradient(p, f0, run["dt"], steps, inner, scheme | W.MIXED, None,
                                   fields=True)
    Lf, *gf, ff = adjoint_gradient(p, f0, run["dt"], steps, inner, scheme, None, fields=True)
    print(f"L mixed {Lm:.15e} fp64 {Lf:.15e}", flush=True)
    assert abs(Lm - Lf) <= 1e-6 * abs(Lf)
    for nm, a, b in zip(["u0", "v0", "p0", "T0"], fm, ff):
        d = normdiff(a, b)
        print(f"combined gradient {nm}: max|g| {np.abs(b).max():.3e}, rel {d:.2e}", flush=True)
        assert np.abs(b).max() > 0
        assert np.isfinite(a).all()
        assert d <= TOL_MIXED, (nm, d)


def test_mixed_forward_adjoint_combined_configured_run(sts_mod):
    # the configured combined run: 500 steps x 10 passes, sqrt(N) checkpoints
    # (23 steps a segment); every parameter and initial-state gradient of the
    # mixed forward against the FP64 forward's (in 500 steps the drag does
    # not feel the inlet 1126 cells upstream: that gradient is 0 in both)
    p, run = W.workload("combined_4096x1024")
    f0 = W.initial_fields(p, run["seed"])
    steps, inner, scheme = run["steps"], run["inner"], W.EXPLICIT | W.TVD
    print(f"case combined 4096x1024 {steps}x{inner} mixed forward vs fp64", flush=True)
    Lm, gu_m, g0_m, g1_m, fm = adjoint_gradient(p, f0, run["dt"], steps, inner,
                                                 scheme | W.MIXED, None, fields=True)
    Lf, gu_f, g0_f, g1_f, ff = adjoint_gradient(p, f0, run["dt"], steps, inner, scheme, None,
                                                 fields=True)
    print(f"L mixed {Lm:.15e} fp64 {Lf:.15e}", flush=True)
    assert abs(Lm - Lf) <= 1e-6 * abs(Lf)
    assert not gu_f.any() and not gu_m.any(), (np.abs(gu_f).max(), np.abs(gu_m).max())
    for nm, a, b in zip(["wall_T0", "wall_T1", "u0", "v0", "p0", "T0"],
                        [g0_m, g1_m, *fm], [g0_f, g1_f, *ff]):
        d = normdiff(a, b)
        print(f"combined gradient {nm}: max|g| {np.abs(b).max():.3e}, rel {d:.2e}", flush=True)
        assert np.abs(b).max() > 0 and np.isfinite(a).all()
        assert d <= TOL_MIXED, (nm, d)
