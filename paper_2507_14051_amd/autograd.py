"""torch.autograd.Function over hlp_unrolled_forward / hlp_unrolled_backward.

    x, y = PDHGUnrolled.apply(c, lc, uc, lv, uv, prob, K, ckpt_every)

runs K iterations of the method on the GPU (controller live in the forward
pass, then frozen) and returns x = D_c xhat_K, y = D_r yhat_K.  The backward
pass is the library's reverse mode over the recorded tape with a checkpoint
every ckpt_every iterations.  Gradients flow to c and the four bound vectors
(infinite bounds get 0); the matrix, its scaling and eta are constants.
"""
from __future__ import annotations

import torch

from .hlp import hlp_tape_bytes, hlp_unrolled_backward, hlp_unrolled_forward


class PDHGUnrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, lc, uc, lv, uv, prob, K, ckpt_every, params=None):
        vecs = [v.detach().to(device=prob.device, dtype=torch.float64).contiguous() for v in (c, lc, uc, lv, uv)]
        prob.update_vectors(*vecs)
        p = prob.params_for(**(params or {}))
        tape = torch.empty(hlp_tape_bytes(prob.handle, K, ckpt_every), dtype=torch.uint8, device=prob.device)
        x = torch.empty(prob.n, dtype=torch.float64, device=prob.device)
        y = torch.empty(prob.m, dtype=torch.float64, device=prob.device)
        hlp_unrolled_forward(prob.handle, p, K, ckpt_every, 0, None, None, x, y, tape)
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
        return gc, glc, guc, glv, guv, None, None, None, None
