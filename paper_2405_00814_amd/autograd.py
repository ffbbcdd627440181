"""torch.autograd.Function over the library's adjoint.

``ProbeEnergyLoss.apply(eps_design, sim, T, window, design, ckpt)`` writes
eps_design (shape (i1-i0, j1-j0)) into the handle's permittivity on the
design box, runs fdtd_adjoint_eps (forward with checkpoints, transposed
layers backward in time) and returns the loss
L = sum_p sum_{m in (n0, n1]} Ez^m[p]^2 as a float64 tensor; backward
returns dL/d eps_design from the same call.  Marshalling only: the forward
and the adjoint both run in the HIP library.
"""
from __future__ import annotations

import torch


class ProbeEnergyLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_design, sim, T, window, design, ckpt_interval=0):
        i0, i1, j0, j1 = design
        assert tuple(eps_design.shape) == (i1 - i0, j1 - j0)
        sim.set_material((i0, j0), (i1, j1), eps_design.detach().float().cpu().numpy())
        loss, grad = sim.adjoint_eps(T, window, design, ckpt_interval)
        ctx.save_for_backward(grad.view(i1 - i0, j1 - j0))
        return torch.tensor(loss, dtype=torch.float64, device=eps_design.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (g * grad.to(g.dtype)).to(torch.float32), None, None, None, None, None


def probe_energy_loss(sim, eps_design, T, window, design, ckpt_interval=0):
    return ProbeEnergyLoss.apply(eps_design, sim, T, window, design, ckpt_interval)
