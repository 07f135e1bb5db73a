"""torch.autograd.Function over the hand-written adjoint of the robust
alignment energy (eq. 2 with the line process eliminated, eq. 4's Psi)."""
import torch

from . import _lib


class AlignLoss(torch.autograd.Function):
    """E = AlignLoss.apply(P_xyz, Q_xyz, corr, coff, T, mu, xi)

    P_xyz (3,NP) / Q_xyz (3,NQ) float32, corr (m,2) int32, coff host int64
    offsets per problem, T (n,4,4) float64 base poses, mu (n,) float64, xi
    (n,6) float64 pose parameters: E is evaluated at the retracted poses
    [Rod(w) | v] T, xi = (w, v) (the retraction of the robust solve).
    Returns E (n,) float64.  Backward gives dE/dP_xyz, dE/dQ_xyz (float32)
    and dE/dxi (float64, the left-perturbation gradient at the retracted pose
    taken through the retraction's Jacobian); T, mu and the correspondences
    get no gradient.  The weights are recomputed, not saved.
    """

    @staticmethod
    def forward(ctx, P_xyz, Q_xyz, corr, coff, T, mu, xi):
        Tx = _lib.se3_retract(xi.to(torch.float64), T)
        ctx.save_for_backward(P_xyz, Q_xyz, corr, Tx, mu, xi)
        ctx.coff = coff
        return _lib.align_loss(P_xyz, Q_xyz, corr, coff, Tx, mu)

    @staticmethod
    def backward(ctx, gE):
        P_xyz, Q_xyz, corr, Tx, mu, xi = ctx.saved_tensors
        dP, dQ, g_left = _lib.align_loss_backward(P_xyz, Q_xyz, corr, ctx.coff, Tx, mu, gE.to(torch.float64))
        dxi = _lib.se3_retract_grad(xi.to(torch.float64), g_left)
        return dP, dQ, None, None, None, None, dxi
