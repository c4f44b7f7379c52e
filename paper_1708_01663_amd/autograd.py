"""Differentiable scattering operator: ``torch.autograd.Function`` over the C ABI.

``scatter(f, op)`` returns the receiver data ``y`` ([T, M], complex) of the
Lippmann-Schwinger forward model at the real contrast ``f`` ([N]); its
backward pass is the vector-Jacobian product of the proof of Prop. 1
(``cisor_vjp``): for the incoming cotangent ``w`` (PyTorch's convention for a
real loss L: ``w = dL/dRe y + i dL/dIm y``) it returns ``Re{J^H w}``.

The backward pass needs the total fields ``u_t`` of the forward solve.  They
are kept according to ``checkpoint``:

* ``"device"``    keep them in GPU memory (fastest);
* ``"host"``      copy them to pinned host memory after the forward pass and
                  back before the backward pass (GPU memory of one field set is
                  only held during the solves);
* ``"recompute"`` keep nothing and solve again in the backward pass, starting
                  from the first-Born field.
"""

from __future__ import annotations

import torch

from .cisor import Cisor, SolveOpts


class _Scatter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, op: Cisor, opts: SolveOpts, checkpoint: str):
        f_ = f.detach().contiguous()
        u, y, _, _ = op.forward(f_, opts)
        ctx.op, ctx.opts, ctx.checkpoint = op, opts, checkpoint
        if checkpoint == "device":
            ctx.u = u
        elif checkpoint == "host":
            host = torch.empty(u.shape, dtype=u.dtype, pin_memory=True)
            host.copy_(u)
            ctx.u = host
            del u
        elif checkpoint == "recompute":
            ctx.u = None
            del u
        else:
            raise ValueError(f"unknown checkpoint mode {checkpoint!r}")
        ctx.save_for_backward(f_)
        return y

    @staticmethod
    def backward(ctx, grad_y):
        (f,) = ctx.saved_tensors
        op = ctx.op
        if ctx.checkpoint == "device":
            u = ctx.u
        elif ctx.checkpoint == "host":
            u = ctx.u.to(op.device, non_blocking=False)
        else:
            u, _, _, _ = op.forward(f, SolveOpts(tol=ctx.opts.tol, maxit=ctx.opts.maxit, start=1,
                                                 replace_every=ctx.opts.replace_every,
                                                 check_every=ctx.opts.check_every), project=False)
        w = grad_y.to(op.cdtype).contiguous()
        g, _, _ = op.vjp(f, u, w, SolveOpts(tol=ctx.opts.tol, maxit=ctx.opts.maxit, start=0,
                                              replace_every=ctx.opts.replace_every,
                                              check_every=ctx.opts.check_every))
        ctx.u = None
        return g.to(f.dtype), None, None, None


def scatter(f, op: Cisor, opts: SolveOpts | None = None, checkpoint: str = "device"):
    """Receiver data y(f) with a backward pass through the adjoint solves."""
    return _Scatter.apply(f, op, opts or SolveOpts(), checkpoint)
