"""Differentiable f(Q) = log det Q + y^T Q^{-1} y for a BTA matrix Q given by its
block arrays (D, B, R, T), the objective of Gaussian (INLA-type) models.

Forward: bta_factor, then bta_solve (x = Q^{-1} y) and bta_logdet_quad, all
enqueued before the factorization's info is read (which raises
NotPositiveDefinite on a failed pivot).
Backward: bta_selinv on the saved factor gives Sigma on the BTA pattern, and
bta_grad_logdet_quad assembles G = Sigma - x x^T on the pattern directly,
scaled by the incoming gradient, with grad_y = 2x.  No dense matrix is formed
and every arithmetic step runs in the HIP library.

Convention: Q is assembled with Q_ii = (D_i + D_i^T)/2, Q_nn = (T + T^T)/2 and
the lower blocks B_i, R_i mirrored into the upper blocks, so
grad_D = G_D, grad_T = G_T, grad_B = 2 G_B, grad_R = 2 G_R.  (The factorization
itself reads only the lower triangles of D and T, so D and T are expected to
be symmetric.)
"""
from __future__ import annotations

import torch

from . import bta


class LogdetQuad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, B, R, T, y):
        LD, LB, LR, LT, info = bta.factor(D.contiguous(), B.contiguous(), R.contiguous(), T.contiguous(), check=False)
        x = bta.solve(LD, LB, LR, LT, y.contiguous())
        f = bta.logdet_quad(LD, LT, y.contiguous(), x)
        # the solve's launches are enqueued while the factorization runs; its
        # outcome is checked once everything is queued (raises on a failed pivot)
        bta.check_info(info)
        ctx.save_for_backward(LD, LB, LR, LT, x)
        return f

    @staticmethod
    def backward(ctx, gf):
        LD, LB, LR, LT, x = ctx.saved_tensors
        X = bta.selinv(LD, LB, LR, LT)
        scale = gf.detach().to(dtype=torch.float64).reshape(()).contiguous()
        GD, GB, GR, GT, gy = bta.grad_logdet_quad(X, x, scale=scale, out=X, want_gy=ctx.needs_input_grad[4])
        return GD, GB, GR, GT, gy


def logdet_quad(D, B, R, T, y):
    """f = log det Q + y^T Q^{-1} y (differentiable in D, B, R, T and y)."""
    return LogdetQuad.apply(D, B, R, T, y)
