"""torch.autograd.Function over hlp_unrolled_forward / hlp_unrolled_backward.

    x, y = PDHGUnrolled.apply(c, lc, uc, lv, uv, prob, K, ckpt_every[, params, x0, y0])

runs K iterations of the method on the GPU (controller live in the forward
pass, then frozen) from zero or from the warm start (x0, y0) in the original
space, and returns x = D_c xhat_K, y = D_r yhat_K.  The backward
pass is the library's reverse mode over the recorded tape with a checkpoint
every ckpt_every iterations.  Gradients flow to c and the four bound vectors
(infinite bounds get 0); the matrix, its scaling, eta and the warm start
are constants.
"""
from __future__ import annotations

import torch

from .hlp import hlp_tape_bytes, hlp_unrolled_backward, hlp_unrolled_forward


class PDHGUnrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, lc, uc, lv, uv, prob, K, ckpt_every, params=None, x0=None, y0=None):
        vecs = [v.detach().to(device=prob.device, dtype=torch.float64).contiguous() for v in (c, lc, uc, lv, uv)]
        start = []
        for v, size in ((x0, prob.n), (y0, prob.m)):
            if v is not None:
                v = v.detach().to(device=prob.device, dtype=torch.float64).contiguous()
                if v.numel() != size:
                    raise ValueError("warm start has the wrong length")
            start.append(v)
        prob.update_vectors(*vecs)
        p = prob.params_for(**(params or {}))
        tape = torch.empty(hlp_tape_bytes(prob.handle, K, ckpt_every), dtype=torch.uint8, device=prob.device)
        x = torch.empty(prob.n, dtype=torch.float64, device=prob.device)
        y = torch.empty(prob.m, dtype=torch.float64, device=prob.device)
        hlp_unrolled_forward(prob.handle, p, K, ckpt_every, 0, start[0], start[1], x, y, tape)
        ctx.prob = prob
        ctx.tape = tape
        ctx.vecs = vecs
        return x, y

    @staticmethod
    def backward(ctx, gx, gy):
        prob = ctx.prob
        prob.update_vectors(*ctx.vecs)   # the reverse pass uses the forward's vectors
        dev = dict(dtype=torch.float64, device=prob.device)
        gx = None if gx is None else gx.to(**dev).contiguous()
        gy = None if gy is None else gy.to(**dev).contiguous()
        gc, glv, guv = (torch.empty(prob.n, **dev) for _ in range(3))
        glc, guc = (torch.empty(prob.m, **dev) for _ in range(2))
        hlp_unrolled_backward(prob.handle, ctx.tape, gx, gy, gc, glc, guc, glv, guv)
        return gc, glc, guc, glv, guv, None, None, None, None, None, None
