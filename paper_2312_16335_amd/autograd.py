"""torch.autograd wrapper of the projection-loss kernels (argument marshalling only).

``ProjLoss.apply(A, B, Qb, Xb, KQn, KXn, trace_const, lam)`` returns the
scalar sampled-pair + trace loss of lv_projloss_fwd; its backward calls
lv_projloss_bwd on the intermediates the forward left in the workspace.
``refine`` runs Adam steps with projection onto the spectral-norm ball.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as lv


class ProjLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, Qb, Xb, KQn=None, KXn=None, trace_const=0.0, lam=1.0):
        A, B, Qb, Xb = (t.contiguous() for t in (A, B, Qb, Xb))
        d, D = A.shape
        ws = torch.empty(lv.lv_projloss_workspace_size(Qb.shape[0], Xb.shape[0], D, d),
                         dtype=torch.uint8, device=A.device)
        loss = torch.empty(3, dtype=torch.float32, device=A.device)
        lv.lv_projloss_fwd(A, B, Qb, Xb, loss, ws, KQn, KXn, trace_const, lam)
        ctx.save_for_backward(A, B, Qb, Xb)
        ctx.extra = (ws, KQn, KXn, lam)
        ctx.parts = loss
        return loss[0].clone()

    @staticmethod
    def backward(ctx, grad):
        A, B, Qb, Xb = ctx.saved_tensors
        ws, KQn, KXn, lam = ctx.extra
        dA = torch.empty_like(A)
        dB = torch.empty_like(B)
        # grad is a device scalar; the kernels take the scale on the host
        lv.lv_projloss_bwd(A, B, Qb, Xb, dA, dB, ws, KQn, KXn, lam, float(grad.item()))
        return dA, dB, None, None, None, None, None, None


def refine(A0: np.ndarray, B0: np.ndarray, sample_block, steps: int, lr: float = 1e-3,
           KQn=None, KXn=None, trace_const: float = 0.0, lam: float = 1.0, device="cuda",
           callback=None):
    """Adam on (A, B) with the projection onto C after each step (device Gram matrix and
    factor application, host float64 eigendecomposition)."""
    A = torch.tensor(A0, dtype=torch.float32, device=device)
    B = torch.tensor(B0, dtype=torch.float32, device=device)
    mA, vA = torch.zeros_like(A), torch.zeros_like(A)
    mB, vB = torch.zeros_like(B), torch.zeros_like(B)
    d, D = A.shape
    ws = None
    loss = torch.empty(3, dtype=torch.float32, device=device)
    dA, dB = torch.empty_like(A), torch.empty_like(B)
    cws = torch.empty(lv.lv_clip_spectral_device_workspace_size(d, D), dtype=torch.uint8,
                      device=device)
    for t in range(1, steps + 1):
        Qb, Xb = sample_block(t)
        if ws is None:
            ws = torch.empty(lv.lv_projloss_workspace_size(Qb.shape[0], Xb.shape[0], D, d),
                             dtype=torch.uint8, device=device)
        lv.lv_projloss_fwd(A, B, Qb, Xb, loss, ws, KQn, KXn, trace_const, lam)
        lv.lv_projloss_bwd(A, B, Qb, Xb, dA, dB, ws, KQn, KXn, lam, 1.0)
        lv.lv_adam_step(A, dA, mA, vA, lr, t)
        lv.lv_adam_step(B, dB, mB, vB, lr, t)
        lv.lv_clip_spectral_device(A, cws)
        lv.lv_clip_spectral_device(B, cws)
        if callback is not None:
            callback(t, loss)
    return A.double().cpu().numpy(), B.double().cpu().numpy()
