"""torch.autograd binding of the hand-written adjoint.

``abc_objective(solver, psi0, V, n_steps, objective)`` returns J(psi_N) as a
0-d float64 tensor; its backward calls the library's reverse-mode adjoint
(checkpointed), so gradients flow to psi0 and V and from there, through
ordinary torch operations, to whatever parameters built them (well amplitude
and centre, packet momentum).  The forward value comes from the same adjoint
call's forward sweep, so one call serves both passes when gradients are
needed; when neither psi0 nor V requires a gradient, only the forward steps
and the objective run.
"""
from __future__ import annotations

import torch


class AbcObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, V, solver, n_steps, objective, ckpt_stride):
        psi0c = psi0.detach().contiguous()
        Vc = None if V is None else V.detach().contiguous()
        if not any(ctx.needs_input_grad[:2]):
            # no gradient asked for: the forward steps and the objective only
            return torch.tensor(solver.objective(psi0c, Vc, n_steps, objective), dtype=torch.float64,
                                device=psi0.device)
        J, gpsi, gV = solver.adjoint(psi0c, Vc, n_steps, objective, ckpt_stride)
        ctx.save_for_backward(gpsi, gV)
        ctx.has_V = V is not None
        return torch.tensor(J, dtype=torch.float64, device=psi0.device)

    @staticmethod
    def backward(ctx, gJ):
        gpsi, gV = ctx.saved_tensors
        return gJ * gpsi, (gJ * gV if ctx.has_V else None), None, None, None, None


def abc_objective(solver, psi0, V, n_steps, objective="prob", ckpt_stride=0):
    """J after n_steps with gradients through the library's adjoint."""
    return AbcObjective.apply(psi0, V, solver, n_steps, objective, ckpt_stride)
