"""The three-dimensional step on the GPU (sts3_* through the C ABI) against
the FP64 3-D oracle (oracle/ora3.c).

Asserted: normwise relative difference <= 1e-10 per field (max |a - b| /
max |b|) and the residuals (the kernels evaluate the equations in other
operation orders, with fused multiply-adds, so the two agree to rounding).
Implicit TVD is compared step by step from shared states (its limiter ties
let rounding-level differences grow over many steps, as in the 2-D parity
tests).  Cases: the small duct in every scheme; a periodic box with
stretched widths, a body force and a random state; walls in y and z of both
types with moving walls on a ragged grid (extents not multiples of the
64 x 4 thread blocks); one step of the mid-size duct from a GPU-advanced
state; one configured step of the large duct (the benchmark's workload and
launch configuration) from a GPU-advanced state, every field; the uniform
stream; argument checks.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1802_04243_amd import workloads3 as W3

pytestmark = pytest.mark.gpu

SCHEMES = {"explicit_upwind": 0, "explicit_tvd": 2, "implicit_upwind": 1, "implicit_tvd": 3}
TOL = 1e-10


@pytest.fixture(scope="module")
def sts3_mod():
    import torch
    assert torch.cuda.is_available()
    from paper_1802_04243_amd import sts3
    return sts3


@pytest.fixture(scope="module")
def ora3():
    from oracle import oracle3
    return oracle3


def normdiff(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def compare(g, o, label, tol=TOL):
    errs = [normdiff(a, b) for a, b in zip(g.fields(), o.fields())]
    rg, ro = g.residuals(), o.residuals()
    print(f"{label}: fields " + " ".join(f"{n}={e:.2e}" for n, e in zip("uvwpT", errs)) +
          f" | residuals gpu {rg[:5].max():.3e} oracle {ro[:5].max():.3e}", flush=True)
    assert max(errs) <= tol, (label, errs)
    scale = max(np.abs(ro[:5]).max(), 1e-300)
    assert np.abs(rg[:5] - ro[:5]).max() <= 1e-8 * scale + 1e-14, (rg, ro)
    assert abs(rg[5] - ro[5]) <= 1e-6 * abs(ro[5]) + 1e-13, (rg[5], ro[5])
    return errs


def run_pair(sts3_mod, ora3, box, f0, dt, steps, inner, scheme, label):
    resync = scheme == 3
    print(f"case {label} scheme={scheme} grid={box.n} steps={steps}x{inner}"
          f"{' (step by step from shared states)' if resync else ''}", flush=True)
    g, o = sts3_mod.Solver3(box), ora3.Oracle3(box)
    g.set_fields(*f0)
    o.set_fields(*f0)
    for s in range(steps):
        if resync and s:
            o.set_fields(*g.fields())
        g.step(dt, inner, scheme)
        o.step(dt, inner, scheme)
        if resync:
            compare(g, o, f"{label} step {s + 1}")
    if not resync:
        compare(g, o, label)
    g.close()


@pytest.mark.parametrize("name,scheme", list(SCHEMES.items()))
def test_duct_60x12x12(sts3_mod, ora3, name, scheme):
    b, run = W3.workload3("duct_60x12x12")
    run_pair(sts3_mod, ora3, b, W3.initial_fields3(b, run["seed"]), run["dt"], 8, run["inner"],
             scheme, f"duct_60x12x12/{name}")


def _random_state(box, seed, base_u=0.3):
    rng = np.random.default_rng(seed)
    f = [0.1 * rng.normal(size=s) for s in box.shapes()]
    f[0] += base_u
    f[3] = 1.0 + 0.05 * rng.uniform(-1, 1, f[3].shape)
    f[4] = 1.0 + 0.05 * rng.uniform(-1, 1, f[4].shape)
    return f


@pytest.mark.parametrize("name,scheme", list(SCHEMES.items()))
def test_periodic_box_stretched(sts3_mod, ora3, name, scheme):
    rng = np.random.default_rng(21)
    box = W3.Box3(d=(rng.uniform(0.05, 0.12, 21), rng.uniform(0.05, 0.12, 10),
                     rng.uniform(0.05, 0.12, 7)), bc=(W3.PERIODIC,) * 3, Ma=0.6, Re=15.0,
                  g=(0.3, -0.2, 0.1))
    run_pair(sts3_mod, ora3, box, _random_state(box, 22), 0.004, 4, 8, scheme,
             f"periodic 21x10x7/{name}")


@pytest.mark.parametrize("name,scheme", list(SCHEMES.items()))
def test_walls_of_both_types_ragged(sts3_mod, ora3, name, scheme):
    rng = np.random.default_rng(31)
    box = W3.Box3(d=(rng.uniform(0.05, 0.12, 67), rng.uniform(0.05, 0.12, 13),
                     rng.uniform(0.05, 0.12, 9)), bc=(W3.PERIODIC, W3.WALLS, W3.WALLS),
                  wall_type=((W3.NOSLIP, W3.NOSLIP), (W3.NOSLIP, W3.SLIP), (W3.SLIP, W3.NOSLIP)),
                  wall_vel=(((0, 0, 0), (0, 0, 0)), ((0.3, 0, -0.2), (0, 0, 0)),
                            ((0, 0, 0), (-0.1, 0.25, 0))),
                  wall_T=((1, 1), (1.2, 1.0), (1.0, 0.85)), Ma=0.9, Re=12.0, g=(0.2, -0.3, 0.4))
    run_pair(sts3_mod, ora3, box, _random_state(box, 32), 0.003, 4, 8, scheme,
             f"walls 67x13x9/{name}")


@pytest.mark.parametrize("name,scheme", list(SCHEMES.items()))
def test_duct_160x32x32_step_from_gpu_state(sts3_mod, ora3, name, scheme):
    b, run = W3.workload3("duct_160x32x32")
    print(f"case duct_160x32x32/{name}: 3 GPU steps, then one step on both", flush=True)
    g, o = sts3_mod.Solver3(b), ora3.Oracle3(b)
    g.set_fields(*W3.initial_fields3(b, run["seed"]))
    for _ in range(3):
        g.step(run["dt"], run["inner"], scheme)
    o.set_fields(*g.fields())
    g.step(run["dt"], run["inner"], scheme)
    o.step(run["dt"], run["inner"], scheme)
    compare(g, o, f"duct_160x32x32/{name}")
    g.close()


@pytest.mark.parametrize("name,scheme", [("explicit_upwind", 0), ("explicit_tvd", 2)])
def test_duct_512x128x128_step_from_gpu_state(sts3_mod, ora3, name, scheme):
    # 8.4M cells, 10 passes: the grids of every launch as the benchmark runs
    # them; the oracle takes about 15 s per step here
    b, run = W3.workload3("duct_512x128x128")
    print(f"case duct_512x128x128/{name}: 1 GPU step, then one step on both", flush=True)
    g, o = sts3_mod.Solver3(b), ora3.Oracle3(b)
    g.set_fields(*W3.initial_fields3(b, run["seed"]))
    g.step(run["dt"], run["inner"], scheme)
    o.set_fields(*g.fields())
    g.step(run["dt"], run["inner"], scheme)
    o.step(run["dt"], run["inner"], scheme)
    compare(g, o, f"duct_512x128x128/{name}")
    g.close()


def test_uniform_stream_is_preserved(sts3_mod):
    # a uniform stream along x between slip walls: every equation returns its
    # old value up to the rounding of the fused multiply-adds
    box = W3.Box3(d=(np.full(70, 0.1), np.full(9, 0.1), np.full(6, 0.1)),
                  bc=(W3.INLET_OUTLET, W3.WALLS, W3.WALLS), wall_type=((W3.SLIP, W3.SLIP),) * 3,
                  Ma=2.0, Re=20.0)
    for scheme in SCHEMES.values():
        g = sts3_mod.Solver3(box)
        f0 = g.fields()
        g.step(0.01, 5, scheme)
        r = g.residuals()
        print(f"uniform stream scheme {scheme}: residuals {r}", flush=True)
        assert np.all(np.abs(r) <= 1e-14), r
        for a, b in zip(g.fields(), f0):
            assert np.abs(a - b).max() <= 1e-14
        g.close()


def test_sts3_argument_checks(sts3_mod):
    from paper_1802_04243_amd import sts as S
    b, run = W3.workload3("duct_60x12x12")
    g = sts3_mod.Solver3(b)
    for args in ((0.0, 5, 0), (-1.0, 5, 0), (run["dt"], 0, 0), (run["dt"], 5, 4), (run["dt"], 5, 8)):
        with pytest.raises(S.StsError) as e:
            g.step(*args)
        assert e.value.code == S.STS_EINVAL, args
    with pytest.raises(ValueError):
        g.set_fields(np.zeros((2, 2, 2)))
    g.close()
