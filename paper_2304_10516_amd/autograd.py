"""Differentiable INR evaluation through the C ABI (hand-written backward).

`DVNRFunction.apply(coords, table, weights, model, block)` returns the
normalized INR output of block `block` at `coords` for the table / weight
tensors given; the backward calls the library's encoding scatter and MLP
backward.  Coordinates are not differentiated (the paper trains only the
parameters).  A model trained this way takes the library's fused Adam step by
copying the gradients into the handle's gradient buffer and calling
`model.adam_step()`.
"""
from __future__ import annotations

import torch


class DVNRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, table, weights, model, block=0):
        coords = coords.contiguous()
        table = table.contiguous()
        weights = weights.contiguous()
        feats = model.encode_forward(coords, table, block=block)
        out = model.mlp_forward(feats, weights, block=block)
        ctx.save_for_backward(coords, table, weights, feats)
        ctx.model = model
        ctx.block = block
        return out

    @staticmethod
    def backward(ctx, dout):
        coords, table, weights, feats = ctx.saved_tensors
        model = ctx.model
        dout = dout.contiguous()
        dweights = torch.zeros_like(weights)
        dfeats = model.mlp_backward(feats, weights, dout, dweights, block=ctx.block)
        dtable = torch.zeros_like(table)
        model.encode_backward(coords, dfeats, dtable, block=ctx.block)
        return None, dtable, dweights, None, None


def inr(coords, table, weights, model, block=0):
    return DVNRFunction.apply(coords, table, weights, model, block)
