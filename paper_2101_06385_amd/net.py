"""PyTorch autograd wrapper of the generalized-SP2 network of libsp2.

SP2Net holds K trainable FP32 triples (W_k, B_k, c_k) of the layers
X_{k+1} = W_k X_k^2 + B_k X_k + c_k I (Eq. general SP2 applied to matrices).  Forward and
backward are the library's HIP kernels (sp2_net_forward / sp2_net_backward); PyTorch only
holds the tensors and the autograd graph.
"""
from __future__ import annotations

import torch

from . import sp2


class SP2NetFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, w, b, c, precision, ckpt_every):
        x0 = x0.contiguous()
        w, b, c = w.contiguous(), b.contiguous(), c.contiguous()
        xk, ws = sp2.net_forward(x0, w, b, c, precision, ckpt_every)
        ctx.save_for_backward(w, b, c)
        ctx.ws = ws
        ctx.precision = precision
        ctx.ckpt_every = ckpt_every
        return xk

    @staticmethod
    def backward(ctx, gk):
        w, b, c = ctx.saved_tensors
        # sp2_net_backward takes the symmetric part of gk itself
        dw, db, dc, g0 = sp2.net_backward(gk.contiguous(), w, b, c, ctx.ws, ctx.precision, ctx.ckpt_every,
                                          want_g0=ctx.needs_input_grad[0])
        return g0, dw, db, dc, None, None


def sp2_branch_init(sigmas):
    """(W, B, c) of truncated SP2 layers: sigma=+1 -> X^2 = (1,0,0), sigma=-1 -> 2X - X^2 = (-1,2,0)."""
    w = torch.tensor([1.0 if s > 0 else -1.0 for s in sigmas], dtype=torch.float32)
    b = torch.tensor([0.0 if s > 0 else 2.0 for s in sigmas], dtype=torch.float32)
    c = torch.zeros(len(sigmas), dtype=torch.float32)
    return w, b, c


class SP2Net(torch.nn.Module):
    def __init__(self, sigmas, precision="fp16x2", ckpt_every=0, device="cuda"):
        super().__init__()
        w, b, c = sp2_branch_init(sigmas)
        self.w = torch.nn.Parameter(w.to(device))
        self.b = torch.nn.Parameter(b.to(device))
        self.c = torch.nn.Parameter(c.to(device))
        self.precision = precision
        self.ckpt_every = ckpt_every

    def forward(self, x0):
        return SP2NetFunction.apply(x0, self.w, self.b, self.c, self.precision, self.ckpt_every)
