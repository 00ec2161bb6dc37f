"""Potential energy as a differentiable torch function.

``LJEnergy.apply(pos, sim)`` returns E = sum_{i<j} V(r_ij) (Eq. LJpotential
with the context's shift) for positions pos (N,3, float64, CUDA).  Its
backward runs the hand-written gradient kernel of the library
(mdpl_lj_backward): dE/dr_i = -F_i (Eq. LJforce), scaled by the incoming
gradient on the device.  The neighbour list is built in forward.
"""
from __future__ import annotations

import torch

from . import mdpl as C
from .sim import LJSim, soa


class LJEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos: torch.Tensor, sim: LJSim):
        x, y, z = soa(pos.detach())
        sim.build(x, y, z)
        _, _, _, pe_w, _ = sim.forces(x, y, z, energy=True)
        ctx.sim = sim
        ctx.save_for_backward(x, y, z)
        return pe_w[0].clone()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        x, y, z = ctx.saved_tensors
        g = grad_out.detach().to(torch.float64).reshape(1).contiguous()
        gx, gy, gz = ctx.sim.backward(x, y, z, g)
        return torch.stack([gx, gy, gz], dim=1), None


def lj_energy(pos: torch.Tensor, sim: LJSim) -> torch.Tensor:
    return LJEnergy.apply(pos, sim)
