"""torch.autograd.Function over ctm_energy_grad (Eq. AD).

The forward pass calls the library once for the energy and its gradient (the
reverse pass runs inside the library, with checkpointed recomputation of the
sweeps); backward only scales the stored gradient by the incoming one.
"""
from __future__ import annotations

import torch


class CTMEnergy(torch.autograd.Function):
    """E = CTMEnergy.apply(A, ctm, n_sweeps, H, terms) for a ``CTM`` context.

    E is the energy per site after ``n_sweeps`` sweeps from the context's
    current environment (held constant); the context's environment is left at
    the result of those sweeps, which makes it a warm start for the next call.
    """

    @staticmethod
    def forward(ctx, A, ctm, n_sweeps, H, terms):
        E, g = ctm.energy_grad(n_sweeps, H, terms, A=A.detach())
        ctx.save_for_backward(g)
        return torch.tensor(E, dtype=torch.float64, device=A.device)

    @staticmethod
    def backward(ctx, gE):
        (g,) = ctx.saved_tensors
        return gE * g, None, None, None, None
