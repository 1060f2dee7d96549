"""torch.autograd.Function around the HIP forward and backward rasteriser.

``render(xy, chol, rgb, W, H)`` returns the [3,H,W] image of Eq. 2 and is
differentiable w.r.t. all three parameter tensors: the forward pass runs
gs2d_project_bin + gs2d_render_fwd, the backward pass gs2d_render_bwd with the
incoming dL/dimg.  Any torch loss can sit on top.
"""
from __future__ import annotations

import torch

from . import _lib


class GS2DRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xy, chol, rgb, W: int, H: int, tile: int = 16, max_pairs=None,
                check_overflow: bool = True):
        xy, chol, rgb = (t.contiguous() for t in (xy, chol, rgb))
        N = xy.shape[0]
        shape = _lib.make_shape(W, H, N, tile, max_pairs)
        ws = _lib.alloc_workspace(shape, xy.device)
        _lib.project_bin(shape, xy, chol, ws)
        if check_overflow:
            st = _lib.read_bins(shape, ws)["status"]
            if st & _lib.STATUS_OVERFLOW:
                raise _lib.GS2DError("gs2d_project_bin", _lib.GS2D_EOVERFLOW)
        img = torch.empty(3, H, W, device=xy.device, dtype=torch.float32)
        _lib.render_fwd(shape, ws, rgb, img=img)
        ctx.shape = shape
        ctx.ws = ws
        ctx.save_for_backward(xy, chol, rgb)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        xy, chol, rgb = ctx.saved_tensors
        N = xy.shape[0]
        g = grad_img.contiguous().to(torch.float32)
        gx = torch.empty(N, 2, device=xy.device)
        gc = torch.empty(N, 3, device=xy.device)
        gr = torch.empty(N, 3, device=xy.device)
        _lib.render_bwd(ctx.shape, ctx.ws, rgb, g, gx, gc, gr)
        return gx, gc, gr, None, None, None, None, None


def render(xy, chol, rgb, W: int, H: int, tile: int = 16, max_pairs=None):
    """Differentiable render of Eq. 2: [3,H,W] FP32."""
    return GS2DRender.apply(xy, chol, rgb, int(W), int(H), int(tile), max_pairs, True)
