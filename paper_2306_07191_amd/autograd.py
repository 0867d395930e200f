"""torch.autograd bridge: the binary32 query (nif_query) as a differentiable
function of an MLP's weights and of the latent grids of the objects that use
it; the backward pass is nif_backward."""
from __future__ import annotations

import torch


class NIFVisibility(torch.autograd.Function):
    """visibility = NIFVisibility.apply(ctx, mlp, rays, ids, tmax, weights, *grids)

    ctx: nif.Context with training buffers (setup_training); weights and grids
    must be the tensors registered in ctx for MLP `mlp` and, in object order,
    for the objects that use it."""

    @staticmethod
    def forward(fctx, ctx, mlp, rays, ids, tmax, weights, *grids):
        ctx.prepare("f32")  # the weights may have changed since the last packing
        y = ctx.query(rays, ids, tmax, dtype="f32")
        fctx.save_for_backward(rays, ids, tmax)
        fctx.nif, fctx.mlp = ctx, mlp
        fctx.objs = [k for k in range(ctx.K) if ctx.mlp_index[k] == mlp]
        return y

    @staticmethod
    def backward(fctx, gy):
        rays, ids, tmax = fctx.saved_tensors
        ctx = fctx.nif
        for k in fctx.objs:
            ctx.train_bufs[k][0].zero_()
        gw = torch.empty(ctx.mlp_params, dtype=torch.float32, device=rays.device)
        ctx.backward(rays, ids, tmax, gy.contiguous().float(), mlp=fctx.mlp, mlp_grad=gw)
        grads = [ctx.train_bufs[k][0].clone() for k in fctx.objs]
        return (None, None, None, None, None, gw, *grads)


def visibility(ctx, rays, ids, tmax, mlp: int = 0):
    """Differentiable visibility of the queries through MLP `mlp`."""
    objs = [k for k in range(ctx.K) if ctx.mlp_index[k] == mlp]
    return NIFVisibility.apply(ctx, mlp, rays, ids, tmax, ctx.mlps[mlp], *[ctx.grids[k] for k in objs])
