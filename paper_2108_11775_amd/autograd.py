"""torch.autograd.Function wrappers over the hand-written occupancy kernels.

OccupancyLogit: s(x; w, beta) forward = the RBF sum kernel; backward = the
hand-written d/dw (Phi^T g) and d/dx (g grad s) kernels.
Occupancy:      c = sigma(s) with the chain through sigma'(s) done in the kernels.
BCEWithLogits:  mean binary cross-entropy on logits and its gradient kernel.
Together they drive the occupancy fit of Sec. 3.1 through autograd, with every
forward and backward step in libpdmp's HIP kernels.
"""
from __future__ import annotations

import torch

from . import Occupancy as _Occ, occupancy_eval, occupancy_bwd, bce_logits


class OccupancyLogit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, weights, hinges, lengthscale):
        occ = _Occ(hinges, weights.detach().contiguous(), float(lengthscale))
        _, s = occupancy_eval(occ, x.detach().contiguous())
        ctx.save_for_backward(x, weights, hinges)
        ctx.lengthscale = float(lengthscale)
        return s

    @staticmethod
    def backward(ctx, g):
        x, weights, hinges = ctx.saved_tensors
        occ = _Occ(hinges, weights.detach().contiguous(), ctx.lengthscale)
        gw, gx = occupancy_bwd(occ, x.detach().contiguous(), g.contiguous(),
                               want_w=ctx.needs_input_grad[1], want_x=ctx.needs_input_grad[0])
        return gx, gw, None, None


class Occupancy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, weights, hinges, lengthscale):
        occ = _Occ(hinges, weights.detach().contiguous(), float(lengthscale))
        c, s = occupancy_eval(occ, x.detach().contiguous())
        ctx.save_for_backward(x, weights, hinges, s)
        ctx.lengthscale = float(lengthscale)
        return c

    @staticmethod
    def backward(ctx, g):
        x, weights, hinges, s = ctx.saved_tensors
        occ = _Occ(hinges, weights.detach().contiguous(), ctx.lengthscale)
        gw, gx = occupancy_bwd(occ, x.detach().contiguous(), g.contiguous(), s_fwd=s,
                               want_w=ctx.needs_input_grad[1], want_x=ctx.needs_input_grad[0])
        return gx, gw, None, None


class BCEWithLogits(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, y):
        s = s.detach().contiguous()
        loss, _ = bce_logits(s, y, want_grad=False)
        ctx.save_for_backward(s, y)
        return loss[0]

    @staticmethod
    def backward(ctx, gout):
        s, y = ctx.saved_tensors
        # the upstream gradient (a device scalar) scales dL/ds inside the kernel
        _, g = bce_logits(s, y, g_scale=gout.detach().contiguous(), want_loss=False)
        return g, None
