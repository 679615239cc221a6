"""Differentiable form: the soft-silhouette loss as a torch.autograd.Function
and the gradient refinement of the CMA-ES mean.

The loss of a candidate theta is the squared-error term of the render loss
(Sec. III-A.2, Eq. (6)) on the soft silhouette computed by tk_soft_forward;
its gradient through the soft raster, the pinhole projection and the forward
kinematics is tk_soft_backward.  This module only marshals arguments; every
step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import tk


class SoftSilhouetteLoss(torch.autograd.Function):
    """loss[b] = sum_p (S_b(p) - M(p))^2 for candidates theta [B, 9 n_arms]
    (FP32, device) of a tracker.Problem.  ws: a workspace from
    tk.soft_workspace(B, ...), reserved for this call until its backward ran."""

    @staticmethod
    def forward(ctx, theta, problem, sigma, ws):
        theta = theta.detach().contiguous()
        B = theta.shape[0]
        xf = torch.empty(B, problem.n_arms, 4, 12, dtype=torch.float32, device=theta.device)
        tk.fk_transform(theta, B, problem.n_arms, problem.chains, xf)
        loss = torch.empty(B, dtype=torch.float64, device=theta.device)
        tk.soft_forward(xf, B, problem.meshes, problem.cam, sigma, problem.target, loss, ws)
        ctx.save_for_backward(theta)
        ctx.problem, ctx.sigma, ctx.ws = problem, sigma, ws
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        (theta,) = ctx.saved_tensors
        p = ctx.problem
        g = torch.empty_like(theta)
        tk.soft_backward(theta, theta.shape[0], p.chains, p.meshes, p.cam, ctx.sigma, g, ctx.ws,
                         grad_loss=grad_loss.contiguous())
        return g, None, None, None


def soft_loss(theta, problem, sigma=1.0, ws=None):
    """Differentiable per-candidate soft-silhouette loss (see SoftSilhouetteLoss)."""
    if ws is None:
        ws = tk.soft_workspace(theta.shape[0], problem.meshes, problem.cam, theta.device)
    return SoftSilhouetteLoss.apply(theta, problem, float(sigma), ws)
