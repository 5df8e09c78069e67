"""Mixed-precision form (scheme bit MIXED): FP32 assembly of the T, u, v
coefficients and FP32 Jacobi corrections applied through an FP64 defect of
each equation; face densities, pressure equation, velocity update, per-step
constants and residuals in FP64.

The form is not bitwise equal to the FP64 method: it moves the coefficients
by FP32 rounding (unit roundoff 2^-24 = 6e-8, about 1 ulp more where the
hardware reciprocal and square root are used).  The tolerances below are
normwise relative differences (max |a - b| / max |b| per field) against the
FP64 oracle or the FP64 GPU path, set above the differences measured on
these cases (a decade for the smooth schemes, about 4x for implicit TVD):

- explicit schemes and implicit upwind: ~6e-8 after 50 x 20 passes at
  120x24, ~2.5e-7 after 20 x 10 passes at 1280x288 and 5120x1152 (largest
  in v, the smallest field) -> 1e-6, and 3e-6 at full size;
- implicit TVD: its limiter multiplies the mass flux in the coefficients and
  jumps where a downstream difference changes sign, so where the FP64 and
  the mixed iterates straddle such a tie the coefficient moves by O(1) and
  the difference no longer scales with the FP32 roundoff: 3.3e-7 at 120x24,
  2.6e-5 (v) at 1280x288, 2.4e-6 at 5120x1152 -> 1e-4, and 3e-4 at full
  size.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {W.EXPLICIT | W.UPWIND: 1e-6, W.EXPLICIT | W.TVD: 1e-6,
       W.IMPLICIT | W.UPWIND: 1e-6, W.IMPLICIT | W.TVD: 1e-4}
TOL_FULL = {k: 3 * v for k, v in TOL.items()}


def normdiff(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def l2diff(a, b):
    den = np.sqrt(np.mean(b * b))
    return float(np.sqrt(np.mean((a - b) ** 2)) / (den if den > 0 else 1.0))


def run_gpu(sts_mod, prob, f0, dt, steps, inner, scheme):
    g = sts_mod.Solver(prob)
    g.set_fields(*f0)
    for _ in range(steps):
        g.step(dt, inner, scheme)
    out = g.fields(), g.residuals()
    g.close()
    return out


def report(label, fm, fr):
    mx = [normdiff(a, b) for a, b in zip(fm, fr)]
    l2 = [l2diff(a, b) for a, b in zip(fm, fr)]
    print(f"{label}: max " + " ".join(f"{n}={e:.2e}" for n, e in zip("uvpT", mx)) +
          " | L2 " + " ".join(f"{n}={e:.2e}" for n, e in zip("uvpT", l2)), flush=True)
    return mx


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_mixed_vs_oracle_120x24(sts_mod, oracle_lib, name, scheme):
    p, run = W.workload("channel_120x24")
    f0 = W.initial_fields(p, run["seed"])
    print(f"case mixed 120x24 {name} {run['steps']}x{run['inner']}", flush=True)
    o = oracle_lib.Oracle(p)
    o.set_fields(*f0)
    for _ in range(run["steps"]):
        o.step(run["dt"], run["inner"], scheme)
    fm, rm = run_gpu(sts_mod, p, f0, run["dt"], run["steps"], run["inner"], scheme | W.MIXED)
    errs = report(f"mixed-vs-oracle 120x24 {name}", fm, o.fields())
    assert all(np.isfinite(a).all() for a in fm)
    assert max(errs) <= TOL[scheme], (name, errs)
    # the mixed form really ran (it is not the FP64 method)
    assert max(errs) > 0.0
    # mass balance of the last pass still holds to FP64 rounding: the
    # continuity residual is assembled in FP64 from the pass's own fluxes
    assert np.isfinite(rm).all()


@pytest.mark.parametrize("name", list(W.SCHEMES))
def test_mixed_vs_oracle_1280x288(sts_mod, oracle_run, name):
    # the configured 200 steps x 10 passes
    scheme = W.SCHEMES[name]
    p, run = W.workload("channel_1280x288")
    f0 = W.initial_fields(p, run["seed"])
    steps = run["steps"]
    print(f"case mixed 1280x288 {name} {steps}x{run['inner']}", flush=True)
    o = oracle_run("channel_1280x288", scheme)
    fm, _ = run_gpu(sts_mod, p, f0, run["dt"], steps, run["inner"], scheme | W.MIXED)
    errs = report(f"mixed-vs-oracle 1280x288 {name}", fm, o.fields())
    assert max(errs) <= TOL[scheme], (name, errs)


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_mixed_vs_fp64_gpu_5120x1152(sts_mod, name, scheme):
    # full size, bench launch configuration: the mixed form against the FP64
    # GPU path (itself within the FP64 parity bar of the oracle on every parity case)
    p, run = W.workload("channel_5120x1152")
    f0 = W.initial_fields(p, run["seed"])
    steps = run["steps"]
    print(f"case mixed 5120x1152 {name} {steps}x{run['inner']}", flush=True)
    fd, _ = run_gpu(sts_mod, p, f0, run["dt"], steps, run["inner"], scheme)
    fm, _ = run_gpu(sts_mod, p, f0, run["dt"], steps, run["inner"], scheme | W.MIXED)
    errs = report(f"mixed-vs-fp64 5120x1152 {name}", fm, fd)
    assert max(errs) <= TOL_FULL[scheme], (name, errs)


def test_mixed_deterministic(sts_mod):
    p, run = W.workload("channel_120x24")
    f0 = W.initial_fields(p, 5)
    a, ra = run_gpu(sts_mod, p, f0, run["dt"], 6, 5, W.IMPLICIT | W.TVD | W.MIXED)
    b, rb = run_gpu(sts_mod, p, f0, run["dt"], 6, 5, W.IMPLICIT | W.TVD | W.MIXED)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(ra, rb)


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_mixed_fused_first_pass_equals_separate_prologue(sts_mod, name, scheme):
    # sts_step runs the prologue inside the first pass; loop 2 with tolerance
    # 0 launches the prologue on its own (the path of the adjoint's
    # recompute): the mixed form must give the same bits either way
    p, run = W.workload("channel_120x24")
    f0 = W.initial_fields(p, 3)
    a, b = sts_mod.Solver(p), sts_mod.Solver(p)
    a.set_fields(*f0)
    b.set_fields(*f0)
    for _ in range(4):
        a.step(run["dt"], 6, scheme | W.MIXED)
        assert b.step_tol(run["dt"], 6, 0.0, scheme | W.MIXED) == 6
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y), name
    a.close()
    b.close()
