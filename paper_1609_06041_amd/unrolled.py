"""Unrolled Algorithm 1 as a ``torch.autograd.Function``.

``unrolled_lowdose(op, b, w, beta, tau, sigma, iters)`` returns x^iters of
exactly ``iters`` APP iterations (Eqs. 18-20) with the given step sizes; the
backward pass is the library's hand-written reverse pass
(``ctpd_unrolled_lowdose_backward``), which recomputes each iteration from its
checkpoint and returns the gradient with respect to b and the scalars beta,
tau, sigma (w is data, not differentiated).  This module only marshals
tensors: both passes run in the HIP library.

``unrolled_lowdose_batch`` runs a list of independent problems, each on its
own operator handle and stream, so that their forward and reverse passes
overlap on the GPU.
"""
from __future__ import annotations

import torch

from . import ctpd


class UnrolledLowdose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, beta, tau, sigma, w, op, iters, tv_iters):
        ckpt = torch.empty(op.ckpt_floats(iters), dtype=torch.float32, device=b.device)
        b = b.detach().contiguous()
        w = w.detach().contiguous()
        vals = (float(beta), float(tau), float(sigma))
        x = op.unrolled_forward(b, w, *vals, iters, ckpt, tv_iters=tv_iters)
        ctx.op, ctx.iters, ctx.tv_iters, ctx.vals = op, iters, tv_iters, vals
        ctx.save_for_backward(b, w, ckpt)
        return x

    @staticmethod
    def backward(ctx, gx):
        b, w, ckpt = ctx.saved_tensors
        gb, (gbeta, gtau, gsigma) = ctx.op.unrolled_backward(b, w, *ctx.vals, ctx.iters, ckpt, gx.contiguous(),
                                                             tv_iters=ctx.tv_iters)
        dev, dt = gx.device, torch.float64
        return (gb, torch.tensor(gbeta, device=dev, dtype=dt), torch.tensor(gtau, device=dev, dtype=dt),
                torch.tensor(gsigma, device=dev, dtype=dt), None, None, None, None)


def unrolled_lowdose(op: ctpd.Operator, b: torch.Tensor, w: torch.Tensor, beta, tau, sigma, iters: int,
                     tv_iters: int = 10) -> torch.Tensor:
    """x^iters of the unrolled Algorithm 1; differentiable in b, beta, tau, sigma
    (pass the scalars as 0-d float64 tensors with requires_grad to get their gradients)."""
    as_t = lambda v: v if isinstance(v, torch.Tensor) else torch.tensor(float(v), dtype=torch.float64)
    return UnrolledLowdose.apply(b, as_t(beta), as_t(tau), as_t(sigma), w, op, int(iters), int(tv_iters))


def unrolled_lowdose_batch(ops, bs, ws, betas, taus, sigmas, iters: int, tv_iters: int = 10):
    """Independent problems, each on its operator's stream (the ops should be
    created on distinct streams so the passes overlap).  Returns the list of x."""
    outs = []
    for op, b, w, be, ta, si in zip(ops, bs, ws, betas, taus, sigmas):
        with torch.cuda.stream(op.stream):
            outs.append(unrolled_lowdose(op, b, w, be, ta, si, iters, tv_iters))
    return outs
