"""torch.autograd wrappers around the hand-written libigr adjoint.

``IGRStep`` is one fixed-dt SSP-RK3 step as an autograd Function: the
forward calls ``igr_step``, the backward calls ``igr_step_adjoint`` (which
recomputes the stage states from the step input inside the library).
Inputs: the padded state U, Sigma, and the jet-disc pressures (a float64
tensor with one entry per disc, on any device); outputs: the new U and
Sigma.  ``run_checkpointed`` chains steps with ``torch.utils.checkpoint``
segments so that only one state per segment is kept between forward and
backward.
"""

from __future__ import annotations

from typing import Callable, Optional

import torch
from torch.utils.checkpoint import checkpoint

from .igr import Solver


class IGRStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U: torch.Tensor, sigma: torch.Tensor, jet_p: torch.Tensor, solver: Solver, dt: float):
        _apply_jet_pressures(solver, jet_p)
        U_out = U.detach().clone()
        S_out = sigma.detach().clone()
        solver.step(U_out, S_out, dt_fixed=dt, sync=False)
        ctx.save_for_backward(U.detach().clone(), sigma.detach().clone(), jet_p.detach().clone())
        ctx.solver = solver
        ctx.dt = dt
        return U_out, S_out

    @staticmethod
    def backward(ctx, U_bar: Optional[torch.Tensor], S_bar: Optional[torch.Tensor]):
        U, sigma, jet_p = ctx.saved_tensors
        solver: Solver = ctx.solver
        _apply_jet_pressures(solver, jet_p)
        if U_bar is None:
            U_bar = torch.zeros_like(U)
        if S_bar is None:
            S_bar = torch.zeros_like(sigma)
        Ub, Sb, pb = solver.step_adjoint(U, sigma, ctx.dt, U_bar.contiguous(), S_bar.contiguous())
        jet_bar = pb[:, 4].to(device=jet_p.device, dtype=jet_p.dtype) if solver.npatch else torch.zeros_like(jet_p)
        return Ub, Sb, jet_bar, None, None


def _apply_jet_pressures(solver: Solver, jet_p: torch.Tensor):
    vals = jet_p.detach().double().cpu().tolist()
    for i, p in enumerate(vals):
        rho, ux, uy, uz, p_old = solver.jets[i]
        if p != p_old:
            solver.set_jet_state(i, rho, ux, uy, uz, p)


def run_checkpointed(solver: Solver, U0: torch.Tensor, sigma0: torch.Tensor, jet_p: torch.Tensor, dt: float,
                     nsteps: int, step_loss: Callable[[torch.Tensor], torch.Tensor], every: int = 10):
    """Advance nsteps fixed-dt steps and return sum_n step_loss(U_n) over
    the states after each step.  Segments of `every` steps are
    checkpointed: their inner states are recomputed during backward."""

    def segment(U, S, p, n):
        loss = U.new_zeros(())
        for _ in range(n):
            U, S = IGRStep.apply(U, S, p, solver, dt)
            loss = loss + step_loss(U)
        return U, S, loss

    U, S = U0, sigma0
    total = U0.new_zeros(())
    done = 0
    while done < nsteps:
        n = min(every, nsteps - done)
        U, S, seg = checkpoint(segment, U, S, jet_p, n, use_reentrant=False)
        total = total + seg
        done += n
    return total, U, S
