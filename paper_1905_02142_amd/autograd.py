"""torch.autograd bindings of the HIP path.

Both functions rebuild the neighbour list from the positions they are given,
so the list is fixed for the forward/backward pair (the descriptor is smooth in
the positions as long as no pair crosses r_cut).  The backward passes run the
library's adjoint kernels; nothing is differentiated by torch itself.

  descriptor(soap, positions, species, cell, pbc)      -> q  (N, K)
      backward: soap_descriptor_grad, the vector-Jacobian product q_bar -> dL/dr
  gap_energy(soap, positions, alpha, species, q_sparse, zeta, cell, pbc) -> E
      E = sum_i sum_s alpha_s (q_i . q_s)^zeta (Sec. III, cohesive energy model);
      backward: dE/dr = -F and dE/dalpha_s from one gap_energy_forces call
"""
from __future__ import annotations

import torch

from .soap import Soap


class _Descriptor(torch.autograd.Function):
    @staticmethod
    def forward(ctx, positions, soap: Soap, species, cell, pbc, struct_offsets):
        nl = soap.neighbors(positions.detach(), cell, pbc, struct_offsets)
        q = soap.descriptor(nl, species)
        ctx.soap, ctx.nl, ctx.species = soap, nl, species
        return q

    @staticmethod
    def backward(ctx, q_bar):
        g = None
        if ctx.needs_input_grad[0]:
            g = ctx.soap.descriptor_grad(ctx.nl, ctx.species, q_bar.contiguous())
        return g, None, None, None, None, None


class _GapEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, positions, alpha, soap: Soap, species, q_sparse, zeta, cell, pbc, struct_offsets):
        nl = soap.neighbors(positions.detach(), cell, pbc, struct_offsets)
        want_f, want_a = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        e, F, ab = soap.energy_forces(nl, species, q_sparse, alpha.detach(), zeta, forces=want_f,
                                      alpha_grad=want_a)
        ctx.save_for_backward(*(t for t in (F, ab) if t is not None))
        ctx.has = (F is not None, ab is not None)
        return e.sum()

    @staticmethod
    def backward(ctx, g):
        saved = list(ctx.saved_tensors)
        F = saved.pop(0) if ctx.has[0] else None
        ab = saved.pop(0) if ctx.has[1] else None
        gpos = -F * g if F is not None else None
        galpha = ab * g if ab is not None else None
        return gpos, galpha, None, None, None, None, None, None, None


def descriptor(soap: Soap, positions: torch.Tensor, species: torch.Tensor, cell, pbc, struct_offsets=None):
    """Normalised power spectrum q of every atom, differentiable in the positions."""
    return _Descriptor.apply(positions, soap, species, cell, pbc, struct_offsets)


def gap_energy(soap: Soap, positions: torch.Tensor, alpha: torch.Tensor, species: torch.Tensor,
               q_sparse: torch.Tensor, zeta: int, cell, pbc, struct_offsets=None):
    """Total GAP energy, differentiable in the positions and in the weights alpha."""
    return _GapEnergy.apply(positions, alpha, soap, species, q_sparse, int(zeta), cell, pbc, struct_offsets)
