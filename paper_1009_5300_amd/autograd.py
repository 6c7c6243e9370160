"""torch.autograd.Function for the total transmission T(V) and its adjoint
gradient dT/dV(r) computed by libiobm (one adjoint solve per outgoing
channel with the same complex-symmetric operator)."""
from __future__ import annotations

import torch

from . import iobm


class Transmission(torch.autograd.Function):
    """T_tot = sum over `energies` and every open incident channel of T_mu.

    forward(V, solver, energies, opts) -> 0-dim float64 tensor; backward
    returns grad_output * dT_tot/dV for V (other inputs get None)."""

    @staticmethod
    def forward(ctx, V, solver, energies, opts=None):
        solver.set_potential(V.detach())
        T, g = solver.grad_transmission(energies, opts)
        ctx.save_for_backward(g)
        return torch.tensor(T, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g.to(grad_out.device), None, None, None


def transmission(V, solver, energies, opts=None):
    return Transmission.apply(V, solver, energies, opts)
