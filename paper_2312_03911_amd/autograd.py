"""torch.autograd bindings of the walk's likelihoods.

The forward pass is `ggns_loglike_grad` without the score; the backward pass is
the hand-written adjoint kernel (`ggns_loglike_vjp`, gx = gout * grad log L),
so differentiating log L needs no framework autodiff.  The likelihood is the
one a run of an `Engine` was configured with (its parameters, precision and,
for matrix-core runs, the BF16-operand definition of the quadratic form).
"""
from __future__ import annotations

import ctypes as C

from . import _lib


def _torch():
    import torch
    return torch


class _LogLike(_torch().autograd.Function):
    @staticmethod
    def forward(ctx, x, engine, run):
        torch = _torch()
        xs = x.detach().to(device=engine.device, dtype=engine._fdtype(run)).contiguous()
        if xs.dim() != 2 or xs.shape[1] != engine.cfgs[run].d:
            raise ValueError(f"x must be [n, {engine.cfgs[run].d}]")
        n = xs.shape[0]
        logl = torch.empty(n, dtype=torch.float64, device=engine.device)
        _lib.check(engine.L.ggns_loglike_grad(engine.ctx, run, C.c_void_p(xs.data_ptr()), n,
                                              C.c_void_p(logl.data_ptr()), None, engine._stream()),
                   "ggns_loglike_grad")
        ctx.engine, ctx.run, ctx.in_dtype = engine, run, x.dtype
        ctx.save_for_backward(xs)
        return logl

    @staticmethod
    def backward(ctx, gout):
        xs, = ctx.saved_tensors
        gx = ctx.engine.loglike_vjp(ctx.run, xs, gout)
        return gx.to(ctx.in_dtype), None, None


def loglike(engine, run: int, x):
    """log L of run `run` at the rows of x ([n, d]); differentiable in x."""
    return _LogLike.apply(x, engine, run)
