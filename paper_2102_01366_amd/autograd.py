"""Differentiation form: N steps of the scheme as a torch.autograd.Function.

The forward pass runs the library's steps with a given time-step sequence
and keeps each step's input state on the device (20 doubles per cell per
step); the backward pass walks the steps in reverse through the library's
discrete adjoint (gks_step_adjoint), which recomputes each step's first
stage from its checkpoint.  The time steps are constants of the map: they
are not differentiated.  This module only sequences library calls.
"""
from __future__ import annotations

import torch


class Rollout(torch.autograd.Function):
    """(W0, gW0) -> (W_N, gW_N) after len(dts) steps of a Solver."""

    @staticmethod
    def forward(ctx, W0, gW0, solver, dts):
        solver.init(W0.detach(), gW0.detach())
        chk = []
        for dt in dts:
            chk.append(solver.read_state(device=True))
            solver.step(float(dt))
        W, gW = solver.read_state(device=True)
        ctx.solver = solver
        ctx.dts = [float(d) for d in dts]
        ctx.chk = chk
        return W, gW

    @staticmethod
    def backward(ctx, Wbar, gWbar):
        s = ctx.solver
        Wb = Wbar.contiguous() if Wbar is not None else torch.zeros((5, s.nc), dtype=torch.float64, device=s.device)
        Gb = gWbar.contiguous() if gWbar is not None else torch.zeros((15, s.nc), dtype=torch.float64, device=s.device)
        for dt, (W, gW) in zip(reversed(ctx.dts), reversed(ctx.chk)):
            Wb, Gb = s.step_adjoint(dt, W, gW, Wb, Gb)
        ctx.chk = None
        return Wb, Gb, None, None


def rollout(solver, W0, gW0, dts):
    """Differentiable N-step map; W0, gW0 are CUDA float64 tensors."""
    return Rollout.apply(W0, gW0, solver, list(dts))


def time_steps(solver, W0, gW0, cfl: float, nsteps: int):
    """The CFL time-step sequence of an undifferentiated run (then held fixed)."""
    solver.init(W0, gW0)
    dts = []
    for _ in range(nsteps):
        dt = solver.compute_dt(cfl)
        solver.step(dt)
        dts.append(dt)
    return dts
