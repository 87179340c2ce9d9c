"""torch.autograd.Function over the fit: per-track chi2 as a differentiable function
of the per-layer alignment (dx, dy, dz, dphi) and material (x/X0).

forward runs kf_fit (seeds from hits) with checkpoints on every ckpt_every-th layer;
backward runs kf_fit_backward, the library's hand-written adjoint, which recomputes the
layers between checkpoints.  Gradients with respect to the hits are not provided.
"""
from __future__ import annotations

import torch


class FitChi2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, align, xX0, hits, hit_mask, kf, ckpt_every=1):
        out = kf.fit(hits, hit_mask, align=align.detach().contiguous(), xX0=xX0.detach().contiguous(), ckpt=True,
                     ckpt_every=ckpt_every)
        ctx.kf = kf
        ctx.fwd = out
        ctx.save_for_backward(align, xX0, hits, hit_mask)
        return out["chi2"]

    @staticmethod
    def backward(ctx, grad_chi2):
        align, xX0, hits, hit_mask = ctx.saved_tensors
        da, dx = ctx.kf.fit_backward(hits, hit_mask, ctx.fwd, grad_chi2.contiguous().float(),
                                     align=align.detach().contiguous(), xX0=xX0.detach().contiguous())
        return da, dx, None, None, None, None


def fit_chi2(kf, hits, hit_mask, align, xX0, ckpt_every=1):
    """Per-track chi2 [n]; differentiable in align [L][4] and xX0 [L].  ckpt_every = k
    keeps the forward's checkpoints on every k-th layer only (memory / k; the backward
    recomputes the rest)."""
    return FitChi2.apply(align, xX0, hits, hit_mask, kf, ckpt_every)
