"""torch.autograd.Function over the expensive ACE-style site energies.

forward(pos) runs the mixed evaluation's geometry (neighbour list, lambda,
buffer, compaction of S) and the expensive forward on S in the HIP library
(`mlmix_compute` with MLMIX_ENERGY_ONLY) and returns the per-atom site energies
E_i (zero outside S). backward(grad_E) calls the hand-written adjoint
(`mlmix_backward`): grad_pos = d(sum_i grad_E_i E_i)/dpos, recomputing the
per-neighbour radial and angular basis instead of storing it. S is frozen at
the forward's value (the derivative of the induced-subsystem energy, as the
force/site-energy relation of the paper's force-mixing section uses it).
"""
import torch

from . import binding as B


class MixedExpensiveEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, system, species, r_buffer=0.0, mode=B.MODE_MIXED):
        pos_d = pos.detach().contiguous()
        out = system.compute(pos_d, species, r_buffer=r_buffer, mode=mode, force_rebuild=True,
                             energy_only=True)
        ctx.system = system
        ctx.generation = system.generation
        ctx.save_for_backward(pos_d, species)
        return out["e_exp"].clone()

    @staticmethod
    def backward(ctx, grad_e):
        pos, species = ctx.saved_tensors
        sy = ctx.system
        if sy.generation != ctx.generation:
            raise RuntimeError("the workspace ran another evaluation after this forward; "
                               "backward needs the forward's dE/dA")
        grad_pos = torch.empty_like(pos)
        sy.backward(pos, species, grad_e.contiguous().to(torch.float64), grad_pos)
        return grad_pos, None, None, None, None


def expensive_energy(pos, system, species, r_buffer=0.0, mode=B.MODE_MIXED):
    """Per-atom expensive site energies, differentiable with respect to pos
    ((3, n) float64 device tensor)."""
    return MixedExpensiveEnergy.apply(pos, system, species, r_buffer, mode)
