"""Gradient of a time-averaged obstacle drag with respect to the inlet
profile and the wall temperatures, through the library's hand-written
adjoint of the explicit-scheme step, as a torch.autograd.Function.

Loss: L = (1/N) sum_{n=1..N} D(state^n), D the drag of sts_drag.  Forward:
N explicit steps from a given initial state (u0, v0, p0, T0), with
checkpoints of the state every `every` steps in device slots.  Backward: for each checkpoint segment,
last first, the segment's states are recomputed from its checkpoint (one
slot per step), then for n = last .. first: lambda += (dL/dD_n) dD/dstate^n
(state^n loaded), state^{n-1} loaded, lambda <- (step n)^T lambda.  The
gradient with respect to u_in is the inlet entries of lambda at the initial
level; the wall-temperature gradients accumulate inside the adjoint steps.
The gradient with respect to the initial state is lambda at the initial
level mapped through the transpose of sts_set_fields' boundary-value
projection, which the library applies (sts_adjoint_read_state_grad).

With scheme bit MIXED the forward (and every recompute) runs the
mixed-precision pass and the backward applies the FP64 step's transpose at
those states.  every=None takes the two-level sqrt(N) schedule: checkpoints
every ceil(sqrt(N)) steps, so that the slots held at once (segment starts
plus the states of one segment) number about 2 sqrt(N).

Every step of the path runs in the library; this module only orders calls.
"""
from __future__ import annotations

import copy
import math
import time
from typing import Sequence

import numpy as np
import torch

from . import sts
from . import workloads as W

# timings and device memory of the last DragLoss evaluation: forward_s,
# backward_s (wall seconds, device synchronised), device_bytes (device
# memory in use at the peak of the backward pass minus before the forward)
LAST_STATS: dict = {}


def _sync():
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def _used() -> int:
    free, total = torch.cuda.mem_get_info()
    return total - free


def _problem(base: W.Problem, u_in, Tw0, Tw1) -> W.Problem:
    p = copy.copy(base)
    p.u_in = np.ascontiguousarray(u_in, dtype=np.float64)
    p.wall_T = (np.ascontiguousarray(Tw0, dtype=np.float64),
                np.ascontiguousarray(Tw1, dtype=np.float64))
    return p


def forward_loss(base: W.Problem, u_in, Tw0, Tw1, f0: Sequence[np.ndarray], dt: float,
                 steps: int, inner: int, scheme: int) -> float:
    """L for given parameters (no checkpoints; used for finite differences)."""
    g = sts.Solver(_problem(base, u_in, Tw0, Tw1))
    g.set_fields(*f0)
    acc = 0.0
    for _ in range(steps):
        g.step(dt, inner, scheme)
        acc += g.drag()
    g.close()
    return acc / steps


class DragLoss(torch.autograd.Function):
    """L(u_in, wall_T[0], wall_T[1], u0, v0, p0, T0) with the adjoint in
    backward()."""

    @staticmethod
    def forward(ctx, u_in, Tw0, Tw1, u0, v0, p0, T0, base, dt, steps, inner, scheme, every):
        if scheme & sts.IMPLICIT:
            raise ValueError("the adjoint is of the explicit scheme")
        if every is None:
            every = max(1, math.ceil(math.sqrt(steps)))
        p = _problem(base, u_in.detach().cpu().numpy(), Tw0.detach().cpu().numpy(),
                     Tw1.detach().cpu().numpy())
        _sync()
        used0 = _used()
        t0 = time.perf_counter()
        g = sts.Solver(p)
        g.set_fields(*[a.detach().cpu().numpy() for a in (u0, v0, p0, T0)])
        ctx.prob = p
        nseg = math.ceil(steps / every)
        g.state_slots(nseg + every)
        acc = 0.0
        for n in range(steps):
            if n % every == 0:
                g.state_save(n // every)
            g.step(dt, inner, scheme)
            acc += g.drag()
        _sync()
        LAST_STATS.clear()
        LAST_STATS.update(forward_s=time.perf_counter() - t0, used0=used0, every=every,
                          slots=nseg + every)
        ctx.g, ctx.meta = g, (dt, steps, inner, scheme, every, nseg)
        ctx.dev = u_in.device
        return torch.tensor(acc / steps, dtype=torch.float64, device=u_in.device)

    @staticmethod
    def backward(ctx, gL):
        g = ctx.g
        dt, steps, inner, scheme, every, nseg = ctx.meta
        w = float(gL) / steps
        _sync()
        t0 = time.perf_counter()
        g.adjoint_begin(inner)
        _sync()
        LAST_STATS["device_bytes"] = _used() - LAST_STATS.get("used0", 0)
        for seg in range(nseg - 1, -1, -1):
            n0, n1 = seg * every, min(steps, (seg + 1) * every)
            # states n0 .. n1-1 of the segment into slots nseg + (n - n0)
            g.state_load(seg)
            for n in range(n0, n1):
                g.state_save(nseg + n - n0)
                g.step(dt, inner, scheme)
            # the current state is level n1
            for n in range(n1, n0, -1):
                if n != n1:
                    g.state_load(nseg + n - n0)
                g.adjoint_seed_drag(w)
                g.state_load(nseg + n - 1 - n0)
                g.adjoint_step(dt, inner, scheme)
        gu, g0, g1 = g.adjoint_read()
        gf = g.adjoint_state_grad()
        LAST_STATS["backward_s"] = time.perf_counter() - t0
        g.close()
        ctx.g = None
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=ctx.dev)  # noqa: E731
        return (t(gu), t(g0), t(g1), *[t(a) for a in gf], None, None, None, None, None, None)


def drag_loss(base: W.Problem, u_in: torch.Tensor, Tw0: torch.Tensor, Tw1: torch.Tensor,
              f0, dt: float, steps: int, inner: int, scheme: int = sts.EXPLICIT,
              every=10) -> torch.Tensor:
    """Time-averaged drag as a differentiable function of (u_in, Tw0, Tw1)
    and of the initial fields f0 = (u0, v0, p0, T0) (numpy arrays or
    tensors; tensors with requires_grad receive the initial-state gradient).
    every: checkpoint interval in steps, or None for ceil(sqrt(steps))."""
    f0 = [a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a), dtype=torch.float64)
          for a in f0]
    return DragLoss.apply(u_in, Tw0, Tw1, *f0, base, dt, steps, inner, scheme, every)
