"""torch.autograd.Function wrappers whose backward passes are the library's
hand-written adjoint kernels.

AcopfEval.apply(x, net)        -> (f [1], c [m])
AcopfBatchEval.apply(x, batch) -> (f [K], c [sum m_k])  (packed layout)

backward(g_f, g_c) returns u = g_f grad f + J' g_c, computed without forming
J (acopf_batch_vjp; a single net uses a cached one-instance batch so that g_f
stays on the device).  That backward is itself differentiable, so double
backward works:
  d/dx    of u along a direction dx = (g_f grad^2 f + sum g_c,r grad^2 c_r) dx
          (Hessian-vector product kernel, H never formed);
  d/dg_c  = J dx (Jacobian-vector product kernel);
  d/dg_f  = grad f . dx (per-instance dot product kernel).
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


def _zeros(n, like):
    return torch.zeros(n, dtype=torch.float64, device=like.device)


class _BatchVjp(torch.autograd.Function):
    """u = w_f grad f + J' w_c for every instance of a batch; differentiable."""

    @staticmethod
    def forward(ctx, x, w_f, w_c, batch):
        x, w_f, w_c = x.contiguous(), w_f.contiguous(), w_c.contiguous()
        u = torch.empty_like(x)
        A.acopf_batch_vjp(batch, x, w_f, w_c, u)
        ctx.save_for_backward(x, w_f, w_c)
        ctx.batch = batch
        return u

    @staticmethod
    def backward(ctx, gu):
        x, w_f, w_c = ctx.saved_tensors
        b = ctx.batch
        gu = gu.contiguous()
        gx = gwf = gwc = None
        if ctx.needs_input_grad[0]:
            gx = torch.empty_like(x)
            A.acopf_batch_hvp(b, x, w_f, w_c, gu, gx)
        if ctx.needs_input_grad[2]:
            gwc = torch.empty_like(w_c)
            A.acopf_batch_jvp(b, x, gu, gwc)
        if ctx.needs_input_grad[1]:
            gf = torch.empty_like(x)
            A.acopf_batch_eval(b, x, None, None, None, gf, None, None, None, A.ACOPF_GRADF)
            gwf = torch.empty_like(w_f)
            A.acopf_batch_xdot(b, gf, gu, gwf)
        return gx, gwf, gwc, None


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
        gf = _zeros(1, x) if gf is None else gf
        gc = _zeros(net.m, x) if gc is None else gc
        return _BatchVjp.apply(x, gf, gc, _one_batch(net)), None


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
        gf = _zeros(b.count, x) if gf is None else gf
        gc = _zeros(int(b.c_off[-1]), x) if gc is None else gc
        return _BatchVjp.apply(x, gf, gc, b), None
