"""torch.autograd.Function wrappers whose backward pass is the library's
hand-written adjoint (VJP) kernel.

AcopfEval.apply(x, net)        -> (f [1], c [m])
AcopfBatchEval.apply(x, batch) -> (f [K], c [sum m_k])  (packed layout)

backward(g_f, g_c) returns u = g_f grad f + J' g_c, computed without
forming J (acopf_batch_vjp; a single net uses a cached one-instance batch
so that g_f stays on the device).  Forward values come from
acopf_eval_f_g / acopf_batch_eval.  Second derivatives are not provided.
"""
from __future__ import annotations

import torch

from . import acopf as A


def _one_batch(net):
    b = getattr(net, "_vjp_batch", None)
    if b is None:
        b = A.acopf_batch_create([net], tile_be=256, grid_mult=0, xcd_group=0, no_graph=1)
        net._vjp_batch = b
    return b


class AcopfEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, net):
        x = x.contiguous()
        f = torch.empty(1, dtype=torch.float64, device=x.device)
        c = torch.empty(net.m, dtype=torch.float64, device=x.device)
        A.acopf_eval_f_g(net, x, f, None, c)
        ctx.save_for_backward(x)
        ctx.net = net
        return f, c

    @staticmethod
    def backward(ctx, gf, gc):
        (x,) = ctx.saved_tensors
        net = ctx.net
        if gf is None:
            gf = torch.zeros(1, dtype=torch.float64, device=x.device)
        if gc is None:
            gc = torch.zeros(net.m, dtype=torch.float64, device=x.device)
        u = torch.empty_like(x)
        A.acopf_batch_vjp(_one_batch(net), x, gf.contiguous(), gc.contiguous(), u)
        return u, None


class AcopfBatchEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, batch):
        x = x.contiguous()
        K = batch.count
        f = torch.empty(K, dtype=torch.float64, device=x.device)
        c = torch.empty(int(batch.c_off[-1]), dtype=torch.float64, device=x.device)
        A.acopf_batch_eval(batch, x, None, None, f, None, c, None, None, A.ACOPF_F | A.ACOPF_C)
        ctx.save_for_backward(x)
        ctx.batch = batch
        return f, c

    @staticmethod
    def backward(ctx, gf, gc):
        (x,) = ctx.saved_tensors
        b = ctx.batch
        if gf is None:
            gf = torch.zeros(b.count, dtype=torch.float64, device=x.device)
        if gc is None:
            gc = torch.zeros(int(b.c_off[-1]), dtype=torch.float64, device=x.device)
        u = torch.empty_like(x)
        A.acopf_batch_vjp(b, x, gf.contiguous(), gc.contiguous(), u)
        return u, None
