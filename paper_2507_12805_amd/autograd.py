"""torch.autograd.Function over the library's dynamic-model op.

Forward and backward run in the HIP kernels behind pmklc_dm_forward /
pmklc_dm_backward (the backward recomputes the activations from the
contexts instead of saving them). Usage:

    logits = DynamicModel.apply(params, ctx, cfg)   # params: flat FP32 (cuda)
    loss = torch.nn.functional.cross_entropy(logits, targets)
    loss.backward()                                  # params.grad from the HIP backward
"""
import torch

from . import dm_backward, dm_forward


class DynamicModel(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, tokens, cfg):
        ctx.save_for_backward(params, tokens)   # inputs only; activations are recomputed
        ctx.cfg = cfg
        return dm_forward(cfg, params, tokens)

    @staticmethod
    def backward(ctx, dlogits):
        params, tokens = ctx.saved_tensors
        grad = dm_backward(ctx.cfg, params, tokens, dlogits.contiguous())
        return grad, None, None
