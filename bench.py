#!/usr/bin/env python3
"""Throughput of the SIMPLE-TS time step on one MI355X.

A step is one full time step of the method on the 5120x1152 channel
(5.9M finite volumes, two squares, Ma 2.43, Re 20): the step prologue, 10
Jacobi passes of loop 2 and the residual reduction (in the FP64 schemes the
prologue runs inside the first pass's launch; the pass roofline is taken
over the other nine).  Inputs are synthetic
(seeded noise on the inlet state) and resident in HBM before timing starts.

Prints one JSON line: MFV-iterations/s (finite volumes x inner passes per
second; the median of three runs of the timed steps), the pass kernel's
achieved bandwidth against the HBM roofline and against a 1 GiB device copy
timed on the same GPU, the FP64 CPU oracle timed on a bounded sample on the
host cores and over the whole configured runs of the 120x24 and 1280x288
channels, and the
mixed-precision form of every scheme (FP32 coefficient assembly and Jacobi
corrections through an FP64 defect): its rate, its speedup over the FP64 form
and its max / L2 relative difference from the FP64 fields after the
configured 200 steps; the four FP64 schemes on the 3000x600 channel and on
the paper's own meshes (4032 x 200 ... 4000, Kn = 0.001, velocity-slip /
temperature-jump walls and square, particle frame); loop 2 run to
convergence (tolerance 1e-6, decided on the device) on the bench workload
against fixed-count steps of the same passes; steps with loop 3 (1, 2, 3
energy-pressure solves per pass) on the bench workload; the
adjoint of the explicit step on the 1024x256 adjoint workload (time-averaged
drag, 100 steps x 10 passes, checkpoints every 10 steps): backward / forward
time and the device memory it holds; and the combined run on the 4096x1024
channel (Re 50, 500 steps x 10 passes): mixed-precision forward, FP64
adjoint, checkpoints every ceil(sqrt(500)) = 23 steps, with its peak device
memory, backward / forward time and the gradient's difference from the one
taken through the FP64 forward.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1802_04243_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_FV_PASS = 96.0       # read u,v,p,T (32) + 4 step constants (32) + write u,v,p,T (32)
HEADLINE = "explicit_tvd"
KERNEL_SOURCES = ["paper_1802_04243_amd/csrc/sts_kernels.hip",
                  "paper_1802_04243_amd/csrc/sts_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pass_kernel_hbm_traffic_5120x1152.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(scheme_name: str):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch", {}).get(scheme_name)


def run_gpu(name: str, steps: int, warmup: int, scheme: int, fields_after: int = 0, f0=None):
    """Timed steps; with fields_after > 0 the run continues (untimed) to that
    many steps in all and returns the fields."""
    import torch
    from paper_1802_04243_amd import sts

    p, run = W.workload(name)
    g = sts.Solver(p)
    g.set_fields(*(f0 if f0 is not None else W.initial_fields(p, run["seed"])))
    dt, inner = run["dt"], run["inner"]
    for _ in range(warmup):
        g.step(dt, inner, scheme)
    g.residuals()
    torch.cuda.synchronize()
    g.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(dt, inner, scheme)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = g.residuals()
    ms, n = g.read_timing()
    g.timing(False)
    for _ in range(warmup + steps, fields_after):
        g.step(dt, inner, scheme)
    fields = g.fields() if fields_after else None
    g.close()
    wall = t1 - t0
    fv_iters = p.n_fv * inner * steps
    pass_ms = ms[1] / max(n[1], 1)
    return dict(wall_s=wall, mfv_iters_s=fv_iters / wall / 1e6, ms_per_step=wall / steps * 1e3,
                # [0]: the prologue, in the FP64 schemes fused with the first pass
                pass_ms=pass_ms, prologue_ms=ms[0] / max(n[0], 1), residual_ms=ms[2] / max(n[0], 1),
                pass_gbs=BYTES_PER_FV_PASS * p.n_fv / (pass_ms * 1e-3) / 1e9,
                residuals=[float(x) for x in res], nx=p.nx, ny=p.ny, dt=dt, inner=inner,
                fields=fields)


def run_loop2(name: str, scheme: int, tol: float, steps: int, warmup: int, max_inner: int = 60):
    """Loop 2 run to convergence (sts_step_tol, decided on the device) against
    the fixed-count step of the same workload: passes per step and time."""
    import torch
    from paper_1802_04243_amd import sts

    p, run = W.workload(name)
    g = sts.Solver(p)
    g.set_fields(*W.initial_fields(p, run["seed"]))
    dt = run["dt"]
    for _ in range(warmup):
        g.step(dt, run["inner"], scheme)
    g.residuals()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = [g.step_tol(dt, max_inner, tol, scheme) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.residuals()
    # the same passes as fixed-count steps, for the per-pass overhead
    t0 = time.perf_counter()
    for k in counts:
        g.step(dt, k, scheme)
    g.residuals()
    torch.cuda.synchronize()
    wall_fixed = time.perf_counter() - t0
    g.close()
    npass = sum(counts)
    return {"workload": name, "tol": tol, "max_inner": max_inner, "steps": steps,
            "passes_per_step": round(npass / steps, 2), "passes_min_max": [min(counts), max(counts)],
            "ms_per_step": round(wall / steps * 1e3, 4), "ms_per_pass": round(wall / npass * 1e3, 5),
            "fixed_count_ms_per_pass": round(wall_fixed / npass * 1e3, 5),
            "mfv_iters_s": round(p.n_fv * npass / wall / 1e6, 2)}


def run_loop3(name: str, scheme: int, steps: int, warmup: int, n3s=(1, 2, 3)):
    """Steps whose passes run loop 3 (n3 energy-pressure solves, sts_step_l3)
    on the bench workload: time per step for each n3."""
    import torch
    from paper_1802_04243_amd import sts

    p, run = W.workload(name)
    out = {"workload": name, "n_inner": run["inner"], "steps": steps}
    for n3 in n3s:
        g = sts.Solver(p)
        g.set_fields(*W.initial_fields(p, run["seed"]))
        for _ in range(warmup):
            g.step_l3(run["dt"], run["inner"], n3, scheme)
        g.residuals()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.step_l3(run["dt"], run["inner"], n3, scheme)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        g.residuals()
        g.close()
        out[f"n3_{n3}"] = {"ms_per_step": round(wall / steps * 1e3, 4),
                           "mfv_iters_s": round(p.n_fv * run["inner"] * steps / wall / 1e6, 2)}
    # loop 2 to convergence (tolerance 1e-6) with one and two solves per pass
    for n3 in (1, 2):
        g = sts.Solver(p)
        g.set_fields(*W.initial_fields(p, run["seed"]))
        for _ in range(warmup):
            g.step(run["dt"], run["inner"], scheme)
        g.residuals()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        counts = [g.step_tol_l3(run["dt"], 60, n3, 1e-6, scheme) for _ in range(5)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        g.close()
        out[f"to_tol_1e-6_n3_{n3}"] = {"passes_per_step": round(sum(counts) / len(counts), 2),
                                       "ms_per_step": round(wall / len(counts) * 1e3, 4)}
    return out


def run_adjoint(name: str = "adjoint_1024x256"):
    """Forward (explicit upwind, drag each step, checkpoints) and backward
    (recompute + hand-written adjoint) of the time-averaged drag loss."""
    import torch
    from paper_1802_04243_amd import adjoint
    p, run = W.workload(name)
    f0 = W.initial_fields(p, run["seed"])
    wb, wt = p.walls()
    for _ in range(2):  # the first run warms the library, its kernels and allocations up
        args = [torch.tensor(a, dtype=torch.float64, requires_grad=True)
                for a in (p.inlet()[0], wb, wt)]
        L = adjoint.drag_loss(p, *args, f0, run["dt"], run["steps"], run["inner"], W.EXPLICIT,
                              run["every"])
        L.backward()
    st = dict(adjoint.LAST_STATS)
    return {"workload": name, "steps": run["steps"], "n_inner": run["inner"],
            "checkpoint_every": run["every"], "scheme": "explicit_upwind",
            "forward_s": round(st["forward_s"], 4), "backward_s": round(st["backward_s"], 4),
            "adjoint_forward_ratio": round(st["backward_s"] / st["forward_s"], 3),
            "device_bytes": int(st["device_bytes"]),
            "note": "forward includes one drag readback per step; backward includes the "
                    "recompute of every checkpoint segment and of every step"}


def _drag_grad(p, f0, run, scheme):
    import torch
    from paper_1802_04243_amd import adjoint
    wb, wt = p.walls()
    args = [torch.tensor(a, dtype=torch.float64, requires_grad=True)
            for a in (p.inlet()[0], wb, wt)]
    ft = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in f0]
    L = adjoint.drag_loss(p, *args, ft, run["dt"], run["steps"], run["inner"], scheme,
                          run["every"])
    L.backward()
    grads = [a.grad.numpy() for a in args + ft]
    return float(L.detach()), grads, dict(adjoint.LAST_STATS)


def run_combined(name: str = "combined_4096x1024", scheme: int = W.EXPLICIT | W.TVD,
                 steps: int = 0):
    """Mixed-precision forward with the FP64 adjoint under sqrt(N)
    checkpoints, and the gradient of the same loss through the FP64 forward
    and adjoint as the reference.  steps > 0 shortens the run (for counter
    collection; the configured run is the default)."""
    p, run = W.workload(name)
    if steps > 0:
        run["steps"] = steps
    f0 = W.initial_fields(p, run["seed"])
    Lm, gm, sm = _drag_grad(p, f0, run, scheme | W.MIXED)
    Lf, gf, sf = _drag_grad(p, f0, run, scheme)
    names = ["u_in", "wall_T0", "wall_T1", "u0", "v0", "p0", "T0"]
    mx, l2 = {}, {}
    for nm, a, b in zip(names, gm, gf):
        den = np.abs(b).max()
        if den == 0:
            continue    # no dependence at FP64 resolution within the horizon
        mx[nm] = float(f"{np.abs(a - b).max() / den:.3e}")
        l2[nm] = float(f"{np.sqrt(np.mean((a - b) ** 2) / np.mean(b * b)):.3e}")
    return {"workload": name, "grid": f"{p.nx}x{p.ny}", "steps": run["steps"],
            "n_inner": run["inner"], "checkpoint_every": sm["every"],
            "checkpoint_slots": sm["slots"], "scheme": "explicit_tvd", "forward": "mixed",
            "forward_s": round(sm["forward_s"], 4), "backward_s": round(sm["backward_s"], 4),
            "adjoint_forward_ratio": round(sm["backward_s"] / sm["forward_s"], 3),
            "peak_device_bytes": int(sm["device_bytes"]),
            "fp64_reference": {"forward_s": round(sf["forward_s"], 4),
                               "backward_s": round(sf["backward_s"], 4),
                               "adjoint_forward_ratio": round(sf["backward_s"] / sf["forward_s"], 3)},
            "loss": Lm, "loss_rel_err_vs_fp64": float(f"{abs(Lm - Lf) / abs(Lf):.3e}"),
            "grad_max_rel_err_vs_fp64": mx, "grad_l2_rel_err_vs_fp64": l2,
            "grad_zero_in_fp64": [nm for nm, b in zip(names, gf) if not np.abs(b).max() > 0]}


def run_other_grid(name: str, steps: int, warmup: int):
    """FP64 throughput of every scheme on another configured grid."""
    out = {}
    p, run = W.workload(name)
    f0 = W.initial_fields(p, run["seed"])
    for nm, sch in W.SCHEMES.items():
        r = run_gpu(name, steps, warmup, sch, f0=f0)
        out[nm] = {"mfv_iters_s": round(r["mfv_iters_s"], 2), "pass_ms": round(r["pass_ms"], 5),
                   "hbm_frac": round(r["pass_gbs"] / HBM_PEAK_GBS, 4),
                   "ms_per_step": round(r["ms_per_step"], 4)}
        print(f"# {name} {nm}: {r['mfv_iters_s']:.1f} MFV-iters/s, pass {r['pass_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    return out


# algorithmic bytes of one 3-D pass per FV: read u, v, w, p, T (40) and the
# five per-step constants C_u, C_v, C_w, C_T, C_p (40), write u, v, w, p, T (40)
BYTES_PER_FV_PASS_3D = 120


def run_three_d(name: str = "duct_512x128x128", steps: int = 5, warmup: int = 2):
    """FP64 throughput of the 3-D step in every scheme: whole steps timed with
    HIP events on the stream the library enqueues on."""
    import torch
    from paper_1802_04243_amd import sts3
    from paper_1802_04243_amd import workloads3 as W3
    b, run = W3.workload3(name)
    f0 = W3.initial_fields3(b, run["seed"])
    out = {"workload": name, "grid": "x".join(str(k) for k in b.n), "n_fv": b.n_fv,
           "steps": steps, "n_inner": run["inner"], "dt": run["dt"],
           "bytes_per_fv_pass_algorithmic": BYTES_PER_FV_PASS_3D}
    for nm, sch in W.SCHEMES.items():
        g = sts3.Solver3(b)
        g.set_fields(*f0)
        for _ in range(warmup):
            g.step(run["dt"], run["inner"], sch)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(steps):
            g.step(run["dt"], run["inner"], sch)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r = g.residuals()
        g.close()
        pass_ms = ms / run["inner"]
        gbs = BYTES_PER_FV_PASS_3D * b.n_fv / (pass_ms * 1e-3) / 1e9
        out[nm] = {"mfv_iters_s": round(b.n_fv * run["inner"] / (ms * 1e-3) / 1e6, 2),
                   "ms_per_step": round(ms, 4), "ms_per_pass_incl_prologue": round(pass_ms, 5),
                   "gbs_algorithmic": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                   "max_residuals": [float(f"{x:.3e}") for x in r[:5]]}
        print(f"# 3-D {name} {nm}: {out[nm]['mfv_iters_s']:.1f} MFV-iters/s, step {ms:.3f} ms",
              file=sys.stderr, flush=True)
    return out


def field_errors(fm, fd):
    """max |a - b| / max |b| and rms(a - b) / rms(b) per field (u, v, p, T)."""
    mx, l2 = {}, {}
    for nm, a, b in zip("uvpT", fm, fd):
        mx[nm] = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
        l2[nm] = float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b * b)), 1e-300))
    return mx, l2


def run_cpu_baseline(name: str, scheme: int, steps: int, threads: int = 0):
    """The FP64 oracle as it stands, on the host cores (all of them, or
    `threads`), on a bounded sample."""
    from oracle import oracle as O
    p, run = W.workload(name)
    o = O.Oracle(p)
    o.set_fields(*W.initial_fields(p, run["seed"]))
    default = O.max_threads()
    if threads:
        O.set_threads(threads)
    cores = O.max_threads()
    try:
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step(run["dt"], run["inner"], scheme)
        t = time.perf_counter() - t0
    finally:
        O.set_threads(default)
    return dict(value=p.n_fv * run["inner"] * steps / t / 1e6, unit="MFV-iters/s", cores=cores,
                kind="oracle",
                sample=f"{steps} step(s) x {run['inner']} passes of {name} ({p.n_fv} FV), "
                       f"{[k for k, v in W.SCHEMES.items() if v == scheme][0]}, {t:.1f} s")


def copy_ceiling(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Bandwidth of a plain 1 GiB device-to-device copy on this GPU (read +
    written bytes per second, GB/s): the achievable ceiling beside the
    datasheet peak.  Timed with events on torch's stream, which runs it."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def run_cpu_whole(name: str, scheme: int):
    """The oracle over a whole configured run (all host threads)."""
    from oracle import oracle as O
    p, run = W.workload(name)
    o = O.Oracle(p)
    o.set_fields(*W.initial_fields(p, run["seed"]))
    t0 = time.perf_counter()
    for _ in range(run["steps"]):
        o.step(run["dt"], run["inner"], scheme)
    t = time.perf_counter() - t0
    return {"mfv_iters_s": round(p.n_fv * run["inner"] * run["steps"] / t / 1e6, 3),
            "seconds": round(t, 2), "run": f"{run['steps']} steps x {run['inner']} passes",
            "cores": O.max_threads()}


def copy_probe(nbytes: int = 1 << 30, reps: int = 3):
    """A plain copy kernel of known size: reads and writes nbytes per launch."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="channel_5120x1152")
    ap.add_argument("--schemes", default="all", help="'all' or a comma list of scheme names")
    ap.add_argument("--cpu-baseline-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision runs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-loop2", action="store_true",
                    help="skip the loop-2-to-convergence timing (sts_step_tol)")
    ap.add_argument("--no-loop3", action="store_true",
                    help="skip the loop-3 timing (sts_step_l3, n3 = 1, 2, 3)")
    ap.add_argument("--no-combined", action="store_true",
                    help="skip the combined run (mixed forward + FP64 adjoint, 4096x1024)")
    ap.add_argument("--other-grids",
                    default="channel_3000x600,paper_4032x200,paper_4032x400,paper_4032x2000,paper_4032x4000",
                    help="comma list of further grids timed with every FP64 scheme ('' = none)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint timing and print its JSON (profiling)")
    ap.add_argument("--combined-only", action="store_true",
                    help="run only the combined run (4096x1024) and print its JSON (profiling)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D step")
    ap.add_argument("--combined-steps", type=int, default=0,
                    help="with --combined-only: steps of a shortened run (counter collection)")
    ap.add_argument("--three-d-only", action="store_true", help="run only the 3-D step")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (counter calibration)")
    a = ap.parse_args()
    if a.copy_probe:
        copy_probe()
        return
    if a.adjoint_only:
        print(json.dumps(run_adjoint()), flush=True)
        return
    if a.combined_only:
        print(json.dumps(run_combined(steps=a.combined_steps)), flush=True)
        return
    if a.three_d_only:
        print(json.dumps(run_three_d()), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    names = list(W.SCHEMES) if a.schemes == "all" else a.schemes.split(",")
    if HEADLINE in names:
        names.remove(HEADLINE)
    names = [HEADLINE] + names
    per, mixed = {}, {}
    # the mixed-form errors are taken after the configured step count
    fields_after = 0 if a.no_mixed else max(W.workload(a.workload)[1]["steps"], a.warmup + a.steps)
    # the headline: the median of three runs of the timed steps
    head_runs = [run_gpu(a.workload, a.steps, a.warmup, W.SCHEMES[HEADLINE]) for _ in range(2)]
    for nm in names:
        per[nm] = run_gpu(a.workload, a.steps, a.warmup, W.SCHEMES[nm], fields_after)
        if nm == HEADLINE:
            head_runs.append(per[nm])
        print(f"# {nm}: {per[nm]['mfv_iters_s']:.1f} MFV-iters/s, pass {per[nm]['pass_ms']:.3f} ms "
              f"({per[nm]['pass_gbs']:.0f} GB/s algorithmic), step {per[nm]['ms_per_step']:.2f} ms",
              file=sys.stderr, flush=True)
        if a.no_mixed:
            continue
        m = run_gpu(a.workload, a.steps, a.warmup, W.SCHEMES[nm] | W.MIXED, fields_after)
        mx, l2 = field_errors(m["fields"], per[nm]["fields"])
        mixed[nm] = {"mfv_iters_s": round(m["mfv_iters_s"], 2),
                     "speedup": round(m["mfv_iters_s"] / per[nm]["mfv_iters_s"], 4),
                     "pass_ms": round(m["pass_ms"], 5),
                     "max_rel_err_vs_fp64": {k: float(f"{v:.3e}") for k, v in mx.items()},
                     "l2_rel_err_vs_fp64": {k: float(f"{v:.3e}") for k, v in l2.items()},
                     "after_steps": fields_after}
        per[nm]["fields"] = m["fields"] = None
        print(f"# {nm}+mixed: {m['mfv_iters_s']:.1f} MFV-iters/s (x{mixed[nm]['speedup']:.3f}), "
              f"max rel err {max(mx.values()):.2e}", file=sys.stderr, flush=True)
    adj = None
    if not a.no_adjoint:
        adj = run_adjoint()
        print(f"# adjoint: forward {adj['forward_s']:.3f} s, backward {adj['backward_s']:.3f} s "
              f"(ratio {adj['adjoint_forward_ratio']:.2f}), device {adj['device_bytes'] / 2**20:.0f} MiB",
              file=sys.stderr, flush=True)
    comb = None
    if not a.no_combined:
        comb = run_combined()
        print(f"# combined: forward {comb['forward_s']:.3f} s, backward {comb['backward_s']:.3f} s "
              f"(ratio {comb['adjoint_forward_ratio']:.2f}), peak {comb['peak_device_bytes'] / 2**30:.2f} GiB, "
              f"grad err {comb['grad_max_rel_err_vs_fp64']}", file=sys.stderr, flush=True)
    loop2 = None
    if not a.no_loop2:
        loop2 = run_loop2(a.workload, W.SCHEMES[HEADLINE], 1e-6, 10, a.warmup)
        print(f"# loop 2 to tol 1e-6: {loop2['passes_per_step']} passes/step, "
              f"{loop2['ms_per_pass']:.4f} ms/pass (fixed count {loop2['fixed_count_ms_per_pass']:.4f})",
              file=sys.stderr, flush=True)
    loop3 = None
    if not a.no_loop3:
        loop3 = run_loop3(a.workload, W.SCHEMES[HEADLINE], 20, a.warmup)
        print("# loop 3: " + ", ".join(f"{k} {v['ms_per_step']:.3f} ms/step" for k, v in loop3.items()
                                      if isinstance(v, dict)), file=sys.stderr, flush=True)
    others = {g: run_other_grid(g, a.steps, a.warmup) for g in a.other_grids.split(",") if g}
    three_d = None if a.no_3d else run_three_d()
    h = sorted(head_runs, key=lambda r: r["mfv_iters_s"])[1]   # the median run
    traffic = measured_traffic(HEADLINE)
    copy_gbs = copy_ceiling()
    roof = dict(bound="hbm", achieved=round(h["pass_gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(h["pass_gbs"] / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel="k_pass (one Jacobi pass)",
                bytes_per_launch=BYTES_PER_FV_PASS * h["nx"] * h["ny"],
                avg_launch_ms=round(h["pass_ms"], 5),
                copy_ceiling_gbs=round(copy_gbs, 1),
                frac_of_copy_ceiling=round(h["pass_gbs"] / copy_gbs, 4))
    cpu = None
    if rank == 0 and not a.no_cpu_baseline:
        cpu = run_cpu_baseline(a.workload, W.SCHEMES[HEADLINE], a.cpu_baseline_steps)
        cpu["value"] = round(cpu["value"], 3)
        cpu["gpu_speedup"] = round(h["mfv_iters_s"] / cpu["value"], 1)
        one = run_cpu_baseline(a.workload, W.SCHEMES[HEADLINE], a.cpu_baseline_steps, threads=1)
        cpu["single_core"] = {"value": round(one["value"], 3), "cores": 1, "sample": one["sample"],
                              "gpu_speedup": round(h["mfv_iters_s"] / one["value"], 1)}
        # whole configured runs: the small parity case and the mid-size grid
        cpu["whole_runs"] = {w: run_cpu_whole(w, W.SCHEMES[HEADLINE])
                             for w in ("channel_120x24", "channel_1280x288")}
    out = {
        "metric": "MFV-iters/s (FP64 SIMPLE-TS step)",
        "value": round(h["mfv_iters_s"], 2),
        "headline_runs": [round(r["mfv_iters_s"], 2) for r in head_runs],
        "unit": "MFV-iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": f"{h['nx']}x{h['ny']}", "scheme": HEADLINE,
                   "n_inner": h["inner"], "dt": h["dt"], "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "schemes": {nm: {"mfv_iters_s": round(r["mfv_iters_s"], 2), "pass_ms": round(r["pass_ms"], 5),
                         "pass_gbs_algorithmic": round(r["pass_gbs"], 1),
                         "hbm_frac": round(r["pass_gbs"] / HBM_PEAK_GBS, 4),
                         "prologue_and_first_pass_ms": round(r["prologue_ms"], 4),
                         "residual_ms": round(r["residual_ms"], 4),
                         "max_residuals": r["residuals"][:5]}
                    for nm, r in per.items()},
        "other_grids": others or None,
        "mixed": mixed or None,
        "loop2_to_convergence": loop2,
        "loop3": loop3,
        "adjoint": adj,
        "combined": comb,
        "three_d": three_d,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
