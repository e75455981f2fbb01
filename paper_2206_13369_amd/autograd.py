"""torch.autograd.Function over K unrolled (multilevel) inexact-ALM iterations.

Forward runs K explicit iterations on the GPU (mlpcp_ialm_step) from S = Y = 0 with a
fixed penalty schedule, keeping (S_k, Y_k) of every iteration as checkpoints.
Backward walks the iterations in reverse; each mlpcp_ialm_step_vjp recomputes its
iteration from the checkpoint and applies the hand-written adjoints of the soft
threshold and of the coarse singular value thresholding.  Gradients flow to D and
lambda; the penalties are constants.
"""
from __future__ import annotations

import torch

from . import ialm_step, ialm_step_vjp, step_workspace


class UnrolledMLPCP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, lam, mus, levels):
        m, n = D.shape
        ws = step_workspace(m, n, levels, D.device)
        lam_f = float(lam)
        S = Y = None
        ckpt = []
        L = None
        ranks = []
        for mu in mus:
            ckpt.append((S, Y))
            L, S, Y, r = ialm_step(D, S, Y, lam_f, mu, levels, workspace=ws)
            ranks.append(r)
        ctx.save_for_backward(D)
        ctx.ckpt = ckpt
        ctx.mus = list(mus)
        ctx.levels = levels
        ctx.lam = lam_f
        ctx.ws = ws
        ctx.ranks = ranks
        return L, S

    @staticmethod
    def backward(ctx, gL, gS):
        (D,) = ctx.saved_tensors
        # the adjoint of D shares D's leading dimension in the C ABI: work on a
        # contiguous D so that both are m x n with ld = n
        D = D.contiguous()
        Db = torch.zeros_like(D)
        Lb = gL.contiguous() if gL is not None else None
        Sb = gS.contiguous() if gS is not None else None
        Yb = None
        lam_b = 0.0
        K = len(ctx.mus)
        for k in range(K - 1, -1, -1):
            S, Y = ctx.ckpt[k]
            Sb, Yb, lb = ialm_step_vjp(D, S, Y, ctx.lam, ctx.mus[k], ctx.levels, Lb, Sb, Yb, Db, workspace=ctx.ws)
            lam_b += lb
            Lb = None   # L_k feeds only its own iteration's S and Y updates
        return Db, torch.tensor(lam_b, dtype=torch.float32, device=D.device), None, None


def unrolled(D, lam, mus, levels: int):
    """(L_K, S_K) of K unrolled iterations, differentiable in D and lam."""
    if not torch.is_tensor(lam):
        lam = torch.tensor(float(lam), dtype=torch.float32, device=D.device)
    return UnrolledMLPCP.apply(D, lam, list(mus), int(levels))
