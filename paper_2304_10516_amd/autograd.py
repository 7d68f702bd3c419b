"""Differentiable INR evaluation through the C ABI (hand-written backward).

`DVNRFunction.apply(coords, table, weights, model)` returns the normalized
INR output at `coords` for the table / weight tensors given; the backward calls
the library's encoding scatter and MLP backward.  Coordinates are not
differentiated (the paper trains only the parameters).
"""
from __future__ import annotations

import torch


class DVNRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, table, weights, model):
        coords = coords.contiguous()
        table = table.contiguous()
        weights = weights.contiguous()
        feats = model.encode_forward(coords, table)
        out = model.mlp_forward(feats, weights)
        ctx.save_for_backward(coords, table, weights, feats)
        ctx.model = model
        return out

    @staticmethod
    def backward(ctx, dout):
        coords, table, weights, feats = ctx.saved_tensors
        model = ctx.model
        dout = dout.contiguous()
        dweights = torch.zeros_like(weights)
        dfeats = model.mlp_backward(feats, weights, dout, dweights)
        dtable = torch.zeros_like(table)
        model.encode_backward(coords, dfeats, dtable)
        return None, dtable, dweights, None


def inr(coords, table, weights, model):
    return DVNRFunction.apply(coords, table, weights, model)
