"""torch.autograd wrappers: the transforms are linear, so each backward is the adjoint.

ZetaFn:   y = Z f,   df = Z^T dy  (px_zeta_adjoint)
MobiusFn: y = M g,   dg = M^T dy  (px_mobius_adjoint)
BatchZetaFn: the same for a batch of posets.
Floating dtypes only (autograd has no integer gradients).
"""

from __future__ import annotations

import torch

from . import poset as _p


class ZetaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, P):
        ctx.P = P
        return _p.zeta(P, f)

    @staticmethod
    def backward(ctx, dy):
        return _p.zeta_adjoint(ctx.P, dy.contiguous()), None


class MobiusFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, P, max_refine=3):
        ctx.P, ctx.max_refine = P, max_refine
        return _p.mobius(P, g, max_refine=max_refine)

    @staticmethod
    def backward(ctx, dy):
        return _p.mobius_adjoint(ctx.P, dy.contiguous(), max_refine=ctx.max_refine), None, None


class BatchZetaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, b):
        ctx.b = b
        return _p.zeta_batched(b, f)

    @staticmethod
    def backward(ctx, dy):
        return _p.zeta_adjoint_batched(ctx.b, dy.contiguous()), None


def zeta_fn(P, f):
    return ZetaFn.apply(f, P)


def mobius_fn(P, g, max_refine=3):
    return MobiusFn.apply(g, P, max_refine)


def batch_zeta_fn(b, f):
    return BatchZetaFn.apply(f, b)
