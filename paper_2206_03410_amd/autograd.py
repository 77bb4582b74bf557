"""torch.autograd wrapper of the library's robust energy and its adjoint.

E(X, V) = E_align + alpha E_reg + beta E_rot (Eq. 4) as a differentiable
function of the node transforms X ([n][4][3], rows A_j^T then t_j^T) and the
source positions V ([N][3]).  The forward pass calls amm_energy_grad, which
evaluates the energy and, in the same launches, the hand-written adjoint
kernels; the backward pass only scales the stored gradients.  Closest points
are those of the evaluation (piecewise constant in X and V) and the
deformation graph (node positions, Eq. (3) weights, Eq. (8) edge weights) is
frozen: only the v_i that appear explicitly in Eq. (2) move with V.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import amm

__all__ = ["RobustEnergy", "robust_energy"]


class RobustEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: torch.Tensor, V: Optional[torch.Tensor], handle, nu_a: float, nu_r: float,
                alpha: float, beta: float):
        if not X.is_cuda:
            raise ValueError("X must be a device tensor")
        if V is not None and (V.dtype != X.dtype or V.device != X.device):
            raise ValueError("V must have X's dtype and device")
        Xc = X.detach().contiguous()
        Vc = V.detach().contiguous() if V is not None else None
        want_x = ctx.needs_input_grad[0]
        want_v = V is not None and ctx.needs_input_grad[1]
        if want_x or want_v:
            gX = torch.empty_like(Xc)
            gV = torch.empty_like(Vc) if want_v else None
            e = amm.amm_energy_grad(handle, Xc, Vc, nu_a, nu_r, alpha, beta, gX, gV)
        else:
            gX = gV = None
            e = amm.amm_energy(handle, Xc, Vc, nu_a, nu_r, alpha, beta)
        ctx.save_for_backward(gX if gX is not None else torch.empty(0, device=X.device),
                              gV if gV is not None else torch.empty(0, device=X.device))
        ctx.has = (want_x, want_v)
        ctx.terms = tuple(e[1:4])
        return torch.tensor(e[0], dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, gE: torch.Tensor):
        gX, gV = ctx.saved_tensors
        want_x, want_v = ctx.has
        dX = gX * gE.to(gX.dtype) if want_x else None
        dV = gV * gE.to(gV.dtype) if want_v else None
        return dX, dV, None, None, None, None, None


def robust_energy(handle, X: torch.Tensor, V: Optional[torch.Tensor] = None, *, nu_a: float,
                  nu_r: float, alpha: float, beta: float) -> torch.Tensor:
    """Differentiable E(X, V) of the problem set on `handle` (V = None: the
    source points given to amm_set_problem, not differentiated).  Returns a
    float64 scalar tensor on X's device."""
    return RobustEnergy.apply(X, V, handle, float(nu_a), float(nu_r), float(alpha), float(beta))
