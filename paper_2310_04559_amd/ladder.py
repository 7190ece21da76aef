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

Scratch comes from PyTorch: unless the caller's options carry a workspace,
each call plans against a budget of half the memory PyTorch could hand out
(at most 128 GiB) and allocates the planned bytes as a tensor, so the caching
allocator serves repeated calls.  The backward never reuses the forward's
workspace: it plans and allocates its own.
"""
from __future__ import annotations

import torch

from . import native

_BUDGET_CAP = 128 << 30


def _budget(device) -> int:
    free, _ = torch.cuda.mem_get_info(device)
    idle = torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
    return int(min(_BUDGET_CAP, (free + max(idle, 0)) // 2))


def _with_workspace(opts, o, v, P, precision, backward, device):
    """``opts`` (or default options) with a PyTorch-allocated workspace that
    holds the library's plan, unless the options already carry one."""
    if opts is not None and opts.workspace:
        return opts
    base = opts if opts is not None else native.make_opts()
    budget = base.hbm_budget or _budget(device)
    nbytes, _ = native.cc_ladder_workspace_query(o, v, P, precision, backward=backward,
                                                 hbm_budget=budget, opts=base)
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    return native.copy_opts(base, workspace=ws)


class LadderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L, t, precision=native.CC_LADDER_FP64, opts=None):
        L = L.contiguous()
        t = t.contiguous()
        R = torch.zeros_like(t)
        P, v, _ = L.shape
        o = t.shape[0]
        run = _with_workspace(opts, o, v, P, native._prec(precision), False, t.device)
        native.cc_ladder_residual(L, t, R, precision, opts=run)
        ctx.save_for_backward(L, t)
        ctx.precision = precision
        ctx.opts = opts
        return R

    @staticmethod
    def backward(ctx, gR):
        L, t = ctx.saved_tensors
        precision = native._prec(ctx.precision)
        if precision in (native.CC_LADDER_SPLIT_BF16, native.CC_LADDER_SPLIT_INT8):
            # the digit forms are forward-only; their adjoint runs in float32
            precision = native.CC_LADDER_FP32
        opts = ctx.opts
        if opts is not None:
            # the forward's workspace is not reused; an upstream gradient need
            # not be pair-symmetric
            opts = native.copy_opts(opts, workspace=None,
                                    flags=opts.flags & ~(native.CC_LADDER_PAIR_SYMMETRIC
                                                         | native.CC_LADDER_CHECK_SYMMETRY
                                                         | native.CC_LADDER_PLUS_MINUS
                                                         | native.CC_LADDER_SYMMETRIC_VECTORS))
        P, v, _ = L.shape
        o = t.shape[0]
        run = _with_workspace(opts, o, v, P, precision, True, t.device)
        dL = torch.zeros_like(L)
        dt = torch.zeros_like(t)
        native.cc_ladder_backward(L, t, gR.contiguous(), dL, dt, precision, opts=run)
        return (dL if ctx.needs_input_grad[0] else None,
                dt if ctx.needs_input_grad[1] else None, None, None)


def ladder(L: torch.Tensor, t: torch.Tensor, precision=native.CC_LADDER_FP64, opts=None):
    return LadderFn.apply(L, t, precision, opts)
