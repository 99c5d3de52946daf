"""Unrolled Algorithm 1 as a ``torch.autograd.Function``.

``unrolled_lowdose(op, b, w, beta, tau, sigma, iters)`` returns x^iters of
exactly ``iters`` APP iterations (Eqs. 18-20) with the given step sizes; the
backward pass is the library's hand-written reverse pass
(``ctpd_unrolled_lowdose_backward``), which recomputes each iteration from its
checkpoint and returns the gradient with respect to b and the scalars beta,
tau, sigma (w is data, not differentiated).  This module only marshals
tensors: both passes run in the HIP library.

``unrolled_lowdose_batch`` runs a list of independent problems, each on its
own operator handle and stream, through the library's many-problem calls, so
that their forward and reverse passes overlap on the GPU.
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


def _fork(main: torch.cuda.Stream, ops) -> None:
    for op in ops:
        if op.stream != main:
            op.stream.wait_stream(main)


def _join(main: torch.cuda.Stream, ops) -> None:
    for op in ops:
        if op.stream != main:
            main.wait_stream(op.stream)


class UnrolledLowdoseMany(torch.autograd.Function):
    """Several independent problems through the library's many-problem calls:
    one host synchronisation per pass for the whole list (two in the reverse
    pass), each problem's kernels on its operator's stream."""

    @staticmethod
    def forward(ctx, ops, ws, iters, tv_iters, betas, taus, sigmas, *bs):
        main = torch.cuda.current_stream()
        bs = [b.detach().contiguous() for b in bs]
        ws = [w.detach().contiguous() for w in ws]
        vals = [t.detach().cpu().tolist() for t in (betas, taus, sigmas)]
        ckpts = [torch.empty(op.ckpt_floats(iters), dtype=torch.float32, device=b.device) for op, b in zip(ops, bs)]
        _fork(main, ops)
        xs = ctpd.unrolled_forward_many(ops, bs, ws, *vals, iters, ckpts, tv_iters=tv_iters)
        _join(main, ops)
        ctx.ops, ctx.iters, ctx.tv_iters, ctx.vals, ctx.P = ops, iters, tv_iters, vals, len(ops)
        ctx.sdev = betas.device
        ctx.save_for_backward(*bs, *ws, *ckpts)
        return tuple(xs)

    @staticmethod
    def backward(ctx, *gxs):
        P = ctx.P
        saved = ctx.saved_tensors
        bs, ws, ckpts = saved[:P], saved[P:2 * P], saved[2 * P:]
        main = torch.cuda.current_stream()
        gxs = [g.contiguous() for g in gxs]
        _fork(main, ctx.ops)
        gbs, g = ctpd.unrolled_backward_many(ctx.ops, bs, ws, *ctx.vals, ctx.iters, ckpts, gxs,
                                             tv_iters=ctx.tv_iters)
        _join(main, ctx.ops)
        g = torch.tensor(g, dtype=torch.float64, device=ctx.sdev)   # P x 3: beta, tau, sigma
        return (None, None, None, None, g[:, 0], g[:, 1], g[:, 2], *gbs)


def unrolled_lowdose_batch(ops, bs, ws, betas, taus, sigmas, iters: int, tv_iters: int = 10):
    """x^iters of independent problems (one operator each; the operators should
    be bound to distinct streams so that their passes overlap).  The scalars
    are sequences of numbers or 0-d float64 tensors (with requires_grad to get
    their gradients).  Returns the list of x, differentiable like
    ``unrolled_lowdose``."""
    def vec(v):
        return torch.stack([a if isinstance(a, torch.Tensor) else torch.tensor(float(a), dtype=torch.float64)
                            for a in v])
    xs = UnrolledLowdoseMany.apply(list(ops), list(ws), int(iters), int(tv_iters), vec(betas), vec(taus),
                                   vec(sigmas), *bs)
    return list(xs)
