"""torch.autograd.Function over the hand-written adjoint of the robust
alignment energy (eq. 2 with the line process eliminated, eq. 4's Psi)."""
import torch

from . import _lib


class AlignLoss(torch.autograd.Function):
    """E = AlignLoss.apply(P_xyz, Q_xyz, corr, coff, T, mu, xi)

    P_xyz (3,NP) / Q_xyz (3,NQ) float32, corr (m,2) int32, coff host int64
    offsets per problem, T (n,4,4) float64, mu (n,) float64, xi (n,6) float64
    a left se(3) perturbation at which the gradient is taken (its value is
    not applied: E is evaluated at T, so dE/dxi is the pose gradient).
    Returns E (n,) float64.  Backward gives dE/dP_xyz, dE/dQ_xyz (float32)
    and dE/dxi (float64); the weights are recomputed, not saved.
    """

    @staticmethod
    def forward(ctx, P_xyz, Q_xyz, corr, coff, T, mu, xi):
        ctx.save_for_backward(P_xyz, Q_xyz, corr, T, mu)
        ctx.coff = coff
        return _lib.align_loss(P_xyz, Q_xyz, corr, coff, T, mu)

    @staticmethod
    def backward(ctx, gE):
        P_xyz, Q_xyz, corr, T, mu = ctx.saved_tensors
        dP, dQ, dxi = _lib.align_loss_backward(P_xyz, Q_xyz, corr, ctx.coff, T, mu, gE.to(torch.float64))
        return dP, dQ, None, None, None, None, dxi
