"""Differentiable SwiftWRF renderer for PyTorch training loops.

The canonical Gaussians and the deformation MLP weights are torch parameters;
every forward pushes them into the library's resident scene
(swf_scene_update) and renders through the HIP path with the per-pixel blend
state kept; the backward calls the hand-written HIP backward
(swf_render_backward). PyTorch only holds the tensors and the stream.
"""
from __future__ import annotations

import torch

from . import binding as B

GAUSSIAN_KEYS = B.PARAMS[:7]


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, tx, flags, *params):
        n_g = len(GAUSSIAN_KEYS)
        gauss = dict(zip(GAUSSIAN_KEYS, params[:n_g]))
        rest = params[n_g:]
        mlp = None
        if rest:
            L = len(rest) // 2
            mlp = (list(rest[:L]), list(rest[L:]))
        renderer.lib.update_scene(renderer.sid, gauss, mlp)
        out, aux = renderer.lib.render(renderer.sid, tx, flags=flags | B.KEEP_AUX,
                                       batch=None if tx is not None else 1)
        ctx.renderer, ctx.flags, ctx.has_mlp = renderer, flags, mlp is not None
        ctx.shapes = [p.shape for p in params]
        ctx.save_for_backward(tx if tx is not None else torch.empty(0), aux)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        tx, aux = ctx.saved_tensors
        r = ctx.renderer
        dev = grad_out.device
        grads = [torch.zeros(s, device=dev, dtype=torch.float32) for s in ctx.shapes]
        n_g = len(GAUSSIAN_KEYS)
        gd = dict(zip(GAUSSIAN_KEYS, grads[:n_g]))
        if ctx.has_mlp:
            L = (len(grads) - n_g) // 2
            gd["weight"] = grads[n_g:n_g + L]
            gd["bias"] = grads[n_g + L:]
        r.lib.render_backward(r.sid, tx if tx.numel() else None, ctx.flags, grad_out.contiguous(), aux, gd)
        return (None, None, None, *grads)


class Renderer(torch.nn.Module):
    """Gaussians (and optionally the deformation MLP) as trainable parameters.

    depth is fixed (it orders the blending and gets no gradient)."""

    def __init__(self, gaussians: dict, H: int, W: int, mlp=None, device: int = 0, lib: B.Context | None = None,
                 room=((0.0, 0.0, 0.0), (6.0, 6.0, 3.0))):
        super().__init__()
        self.lib = lib or B.Context(device)
        self.H, self.W = H, W
        self.sid = self.lib.upload_scene(gaussians, H, W, mlp=mlp, room=room)
        dev = torch.device("cuda", device)
        self.gauss = torch.nn.ParameterList([
            torch.nn.Parameter(torch.as_tensor(gaussians[k], dtype=torch.float32, device=dev).clone())
            for k in GAUSSIAN_KEYS])
        self.weights = torch.nn.ParameterList()
        self.biases = torch.nn.ParameterList()
        if mlp is not None:
            for w in mlp[0]:
                self.weights.append(torch.nn.Parameter(torch.as_tensor(w, dtype=torch.float32, device=dev).clone()))
            for b in mlp[1]:
                self.biases.append(torch.nn.Parameter(torch.as_tensor(b, dtype=torch.float32, device=dev).clone()))

    def forward(self, tx=None, flags: int = 0):
        if len(self.weights) == 0:
            flags |= B.NO_DEFORM
        params = list(self.gauss) + list(self.weights) + list(self.biases)
        return _RenderFn.apply(self, tx, flags, *params)
