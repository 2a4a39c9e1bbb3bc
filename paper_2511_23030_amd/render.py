"""Differentiable rendering as a torch.autograd.Function.

The forward calls ``dcgs_render_fwd`` and keeps its render state; the
backward calls ``dcgs_render_bwd``, the hand-written adjoint that walks each
pixel's list back to front, recovering transmittance by division, and chains
to the raw parameters.  PyTorch only provides device memory and the stream.
"""
from __future__ import annotations

import torch

from . import dcgs as D


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, lib_ctx, cam, bg, sh_degree, tile):
        if params.dim() != 2 or params.stride(1) != 1:
            raise ValueError("params must be a [R, n] tensor with contiguous rows")
        st = D.RenderState(lib_ctx)
        n = params.shape[1]
        rgb, depth = st.forward(params.detach(), n, sh_degree, cam, bg, tile)
        fctx.st = st
        fctx.save_for_backward(params)
        fctx.mark_non_differentiable()
        return rgb, depth

    @staticmethod
    def backward(fctx, g_rgb, g_depth):
        (params,) = fctx.saved_tensors
        n = params.shape[1]
        g_rgb = torch.zeros_like(params[:0]) if g_rgb is None else g_rgb.contiguous()
        g_depth = None if g_depth is None else g_depth.contiguous()
        grad = torch.empty(params.shape[0], max(n, 1), dtype=params.dtype, device=params.device)
        fctx.st.backward(params.detach(), n, g_rgb, g_depth, grad)
        fctx.st.close()
        return grad[:, :n], None, None, None, None, None


def render(params: torch.Tensor, lib_ctx: D.Context, cam: dict, bg=(0.0, 0.0, 0.0),
           sh_degree: int = 3, tile=(16, 16)):
    """RGB [3, H, W] and depth [H, W] of the parameter block `params`
    [R, n] (float32, device), differentiable with respect to params."""
    return _Render.apply(params, lib_ctx, cam, tuple(bg), sh_degree, tuple(tile))
