"""Autograd wrapper of the ladder term.

``ladder(L_vv, t, precision)`` returns a fresh R with
R[i,j,a,b] = sum_cd (sum_x L[x,a,c] L[x,b,d]) t[i,j,c,d]  (eqs. cholesky and
vfunction); its backward calls the library's hand-written adjoint, which
rebuilds the integral blocks instead of storing them.  Gradients are
entrywise in L (no symmetrisation) and need no pair symmetry of the upstream
gradient.  Options carrying the exchange flag give the exchange partner
(eq. vfunction2) and its gradients instead.  The pair-symmetric flag serves the
forward only: the backward clears it, since an upstream gradient need not be
pair-symmetric.
"""
from __future__ import annotations

import torch

from . import native


class LadderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L, t, precision=native.CC_LADDER_FP64, opts=None):
        L = L.contiguous()
        t = t.contiguous()
        R = torch.zeros_like(t)
        native.cc_ladder_residual(L, t, R, precision, opts=opts)
        ctx.save_for_backward(L, t)
        ctx.precision = precision
        ctx.opts = opts
        return R

    @staticmethod
    def backward(ctx, gR):
        L, t = ctx.saved_tensors
        precision = ctx.precision
        if precision == native.CC_LADDER_SPLIT_BF16 or precision == "split_bf16":
            # the slice form is forward-only; its adjoint runs in float32
            precision = native.CC_LADDER_FP32
        opts = ctx.opts
        if opts is not None and opts.flags & native.CC_LADDER_PAIR_SYMMETRIC:
            opts = type(opts).from_buffer_copy(opts)
            opts.flags &= ~native.CC_LADDER_PAIR_SYMMETRIC
        dL = torch.zeros_like(L)
        dt = torch.zeros_like(t)
        native.cc_ladder_backward(L, t, gR.contiguous(), dL, dt, precision, opts=opts)
        return (dL if ctx.needs_input_grad[0] else None,
                dt if ctx.needs_input_grad[1] else None, None, None)


def ladder(L: torch.Tensor, t: torch.Tensor, precision=native.CC_LADDER_FP64, opts=None):
    return LadderFn.apply(L, t, precision, opts)
