"""Velocity-slip / temperature-jump surfaces (eqs pl38, pl39) on the GPU
against the FP64 CPU oracle (through the C ABI).

The FP64 form agrees with the oracle to rounding, as for the other boundary rules;
asserted: normwise relative difference <= 1e-10 per field.  Cases: a small
channel with slip-jump walls moving with the flow and a slip-jump square
(all four schemes, and the mixed-precision form within its FP32 tolerance);
a ragged non-uniform grid mixing wall types, heated walls and a body force;
a periodic channel; one step of every scheme on the paper's 4032x200 mesh
(Kn = 0.001, Ma 2.43, particle frame) from a GPU-advanced state, in the
launch configuration the benchmark times; and the whole 200-step run of
that workload, whose increments must stay bounded.  Plus the argument checks of
the new fields and the drag's rejection of slip-jump obstacles.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1802_04243_amd import workloads as W

from test_parity_gpu import compare, run_pair

pytestmark = pytest.mark.gpu

SJ = W.WALL_SLIP_JUMP


def small_slip_channel():
    x = (np.arange(120) + 0.5) / 120
    return W.Problem(nx=120, ny=24, obstacles=[(57, 9, 62, 14)], wall_type=(SJ, SJ),
                     wall_u=(1.0, 1.0), obstacle_type=SJ, kn=0.01,
                     wall_T=(1.0 + 0.1 * x, 1.05 - 0.1 * x))


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_slip_jump_channel_all_schemes(sts_mod, oracle_lib, name, scheme):
    p = small_slip_channel()
    run_pair(sts_mod, oracle_lib, p, p.cfl_dt(), 30, 10, scheme, 21, label=f"slip-jump 120x24/{name}")


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_slip_jump_mixed_form(sts_mod, oracle_lib, name, scheme):
    p = small_slip_channel()
    f0 = W.initial_fields(p, 21)
    g = sts_mod.Solver(p)
    o = oracle_lib.Oracle(p)
    g.set_fields(*f0)
    o.set_fields(*f0)
    for _ in range(30):
        g.step(p.cfl_dt(), 10, scheme | W.MIXED)
        o.step(p.cfl_dt(), 10, scheme)
    errs = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(g.fields(), o.fields())]
    print(f"slip-jump mixed-vs-oracle {name}: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    g.close()
    assert 0.0 < max(errs) <= (1e-4 if scheme == W.IMPLICIT | W.TVD else 1e-6), errs


@pytest.mark.parametrize("scheme", [W.EXPLICIT | W.TVD, W.IMPLICIT | W.UPWIND])
def test_slip_jump_ragged_mixed_walls(sts_mod, oracle_lib, scheme):
    rng = np.random.default_rng(8)
    nx, ny = 71, 37
    p = W.Problem(nx=nx, ny=ny, dx=rng.uniform(0.03, 0.08, nx), dy=rng.uniform(0.02, 0.05, ny),
                  obstacles=[(20, 5, 26, 12), (40, 20, 43, 36)], wall_type=(SJ, W.WALL_NOSLIP_ISOTHERMAL),
                  wall_u=(0.4, -0.2), wall_T=(rng.uniform(0.9, 1.1, nx), rng.uniform(0.95, 1.2, nx)),
                  obstacle_type=SJ, obstacle_T=1.1, kn=0.004, gx=0.3, gy=-0.1,
                  u_in=W.parabolic_inlet(ny, 3))
    run_pair(sts_mod, oracle_lib, p, p.cfl_dt(), 12, 8, scheme, 5, label="slip-jump ragged")


@pytest.mark.parametrize("scheme", [W.EXPLICIT | W.TVD, W.IMPLICIT | W.TVD])
def test_slip_jump_periodic(sts_mod, oracle_lib, scheme):
    p = W.Problem(nx=67, ny=20, lx=3.0, periodic=True, obstacles=[(30, 7, 35, 12)],
                  wall_type=(SJ, SJ), wall_u=(0.0, 0.5), obstacle_type=SJ, kn=0.02,
                  wall_T=(np.full(67, 1.0), np.linspace(1.0, 1.2, 67)))
    run_pair(sts_mod, oracle_lib, p, 0.01, 12, 8, scheme, 9, label="slip-jump periodic")


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_paper_mesh_4032x200_step_from_gpu_state(sts_mod, oracle_lib, name, scheme):
    p, run = W.workload("paper_4032x200")
    print(f"case paper_4032x200/{name}: 3 GPU steps, then one step on both", flush=True)
    g = sts_mod.Solver(p)
    g.set_fields(*W.initial_fields(p, run["seed"]))
    for _ in range(3):
        g.step(run["dt"], run["inner"], scheme)
    state = g.fields()
    g.set_fields(*state)
    o = oracle_lib.Oracle(p)
    o.set_fields(*state)
    g.step(run["dt"], run["inner"], scheme)
    o.step(run["dt"], run["inner"], scheme)
    compare(g, o, f"paper_4032x200/{name}")
    g.close()


@pytest.mark.parametrize("name,scheme", list(W.SCHEMES.items()))
def test_paper_mesh_4032x200_run_stays_bounded(sts_mod, name, scheme):
    # the workload as the benchmark runs it (200 steps of 10 passes at its
    # time step): loop 2's last-pass increments stay small and finite in
    # every scheme (at twice this time step the explicit TVD run diverges)
    p, run = W.workload("paper_4032x200")
    print(f"case paper_4032x200/{name}: {run['steps']} steps", flush=True)
    g = sts_mod.Solver(p)
    g.set_fields(*W.initial_fields(p, run["seed"]))
    worst = 0.0
    for s in range(run["steps"]):
        g.step(run["dt"], run["inner"], scheme)
        if s % 20 == 19:
            r = g.residuals()   # raises on a non-finite value
            worst = max(worst, r[0], r[1], r[3], r[2] / p.p_in)
    print(f"largest last-pass increment {worst:.2e}", flush=True)
    g.close()
    assert worst < 2e-5, worst


def test_slip_jump_argument_checks(sts_mod):
    import copy
    p = small_slip_channel()
    for field, bad in (("obstacle_type", W.WALL_SLIP_ADIABATIC), ("obstacle_type", 7), ("kn", -1.0),
                       ("kn", float("nan")), ("wall_type", (SJ, 3))):
        q = copy.copy(p)
        setattr(q, field, bad)
        with pytest.raises(sts_mod.StsError) as e:
            sts_mod.Solver(q)
        assert e.value.code == sts_mod.STS_EINVAL, (field, bad)
    g = sts_mod.Solver(p)
    with pytest.raises(sts_mod.StsError) as e:   # the drag is of no-slip surfaces
        g.drag()
    assert e.value.code == sts_mod.STS_EINVAL
    g.close()
