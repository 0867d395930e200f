"""torch.autograd bridge: the binary32 query (nif_query) as a differentiable
function of an MLP's weights and of the latent grids of the objects that use
it; the backward pass is nif_backward.  PaperVisibility does the same for the
paper's outer and inner networks (nif_paper_query / nif_paper_backward)."""
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


class PaperVisibility(torch.autograd.Function):
    """visibility = PaperVisibility.apply(pm, rays, ids, tmax, w_outer, w_inner)

    pm: nif.PaperModel with training buffers for both networks
    (setup_training(0) and (1)); w_outer and w_inner must be the master tensors
    those returned.  The backward returns the gradients of both MLPs and leaves
    the binary32 latent gradients in pm.grid_grad(obj, network)."""

    @staticmethod
    def forward(fctx, pm, rays, ids, tmax, w_outer, w_inner):
        for net in (0, 1):
            pm.set_mlp(net, (w_outer, w_inner)[net].detach())  # the weights may have changed
        pm.prepare("f32")
        y = pm.query(rays, ids, tmax, "f32")
        fctx.save_for_backward(rays, ids, tmax)
        fctx.pm = pm
        return y

    @staticmethod
    def backward(fctx, gy):
        rays, ids, tmax = fctx.saved_tensors
        pm = fctx.pm
        g = gy.contiguous().float()
        grads = []
        for net in (0, 1):
            gw = torch.empty(pm.mlp_params(net), dtype=torch.float32, device=rays.device)
            pm.backward(net, rays, ids, tmax, g, mlp_grad=gw)
            grads.append(gw)
        return (None, None, None, None, grads[0], grads[1])


def paper_visibility(pm, rays, ids, tmax, w_outer, w_inner):
    """Differentiable visibility through the paper's outer and inner networks."""
    return PaperVisibility.apply(pm, rays, ids, tmax, w_outer, w_inner)
