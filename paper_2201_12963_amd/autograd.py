"""torch.autograd entry point for the adjoint gradient of the CPM path.

L(R, dV) = sum_i (q*_i - t_i)^2 + U_coul(R, q*(R, dV)), with q* = S (b(R) + dV c).
The forward call runs cpm_grad, which computes the loss and, by the adjoint
lambda = S [2 (q* - t) + dV c], the gradients with respect to all site
positions and dV in the same pass (the electrolyte charge spectrum of the
forward PPPM step is reused; the mesh of the electrode charges q* - lambda is
recomputed).  backward() only scales them by the incoming gradient.
"""

from __future__ import annotations

import torch


class CPMLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, site_xyz: torch.Tensor, dv: torch.Tensor, q_target: torch.Tensor, cpm):
        loss, dl_dx, dl_ddv, q = cpm.grad(site_xyz.detach().contiguous(), float(dv), q_target.contiguous())
        fctx.save_for_backward(dl_dx, dl_ddv)
        fctx.mark_non_differentiable(q)
        return loss[0], q

    @staticmethod
    def backward(fctx, g_loss, g_q):
        dl_dx, dl_ddv = fctx.saved_tensors
        return g_loss * dl_dx, (g_loss * dl_ddv[0]).reshape(()), None, None


def cpm_loss(cpm, site_xyz: torch.Tensor, dv: torch.Tensor, q_target: torch.Tensor):
    """Differentiable loss (and the charges q*) for a built Context."""
    return CPMLoss.apply(site_xyz, dv, q_target, cpm)
