"""torch.autograd form of the splatting path (one view, K cells).

``render(cells, boxes, camera, settings)`` returns the composed image
(rgb [H,W,3] and transmittance [H,W]) as a differentiable function of every
cell's Gaussian parameters.  Forward = per cell sx_preprocess, sx_sort,
sx_render_partial, then sx_composite (paper Eq. 1-5); backward = sx_backward
(Eq. 6-7 through the composition, each cell's render and projection).  torch
only provides memory and the stream; all arithmetic runs in libsplaxel.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import binding as B
from .pipeline import Frame, GaussianParams


class _SplatFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, frame: Frame, *tensors):
        # every cell enqueued asynchronously; one host synchronisation for
        # the view reads the cells' instance counts back together
        out = frame.forward_checked()
        ctx.frame = frame
        ctx.n_in = len(tensors)
        rgb = out[..., :3]
        T = out[..., 3]
        return rgb.clone(), T.clone()

    @staticmethod
    def backward(ctx, g_rgb, g_T):
        frame: Frame = ctx.frame
        H, W = frame.cam.height, frame.cam.width
        dout = torch.zeros((H, W, 4), dtype=torch.float32, device=frame.out.device)
        if g_rgb is not None:
            dout[..., :3] = g_rgb
        if g_T is not None:
            dout[..., 3] = g_T
        grads = [c.zeros_like() for c in frame.cells]
        frame.backward(dout.contiguous(), grads)
        flat: List[torch.Tensor] = []
        for g in grads:
            flat.extend(g.tensors())
        return (None, *flat)


def render(cells: Sequence[GaussianParams], boxes, camera, settings, flags: int = 0,
           frame: Frame = None):
    """Differentiable render of one view.  Gradients flow to the tensors of
    every GaussianParams in ``cells`` (they should have requires_grad)."""
    if frame is None:
        frame = Frame(cells, boxes, camera, settings, flags=flags)
    tensors = []
    for c in cells:
        tensors.extend(c.tensors())
    return _SplatFn.apply(frame, *tensors)


class Adam:
    """Adam over a list of FP32 tensors with the sx_adam kernel (textbook
    Adam with bias correction; the paper's optimiser is unnamed)."""

    def __init__(self, params: Sequence[torch.Tensor], lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8):
        self.params = list(params)
        self.lr = lr
        self.betas = betas
        self.eps = eps
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    @torch.no_grad()
    def step(self):
        self.t += 1
        for p, m, v in zip(self.params, self.m, self.v):
            if p.grad is None:
                continue
            B.sx_adam(p.data, p.grad.contiguous(), m, v, self.t, self.lr, self.betas[0],
                      self.betas[1], self.eps)

    def zero_grad(self):
        for p in self.params:
            p.grad = None
