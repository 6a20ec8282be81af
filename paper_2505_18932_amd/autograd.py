"""torch.autograd.Function wrappers of the geometry stage.

Both functions call the C ABI for forward and backward; PyTorch only
sequences them and holds the tensors.  Gradients flow to the input depths
(both functions) and to the input colours (splat), never to cameras, the
carried volume or the mask.  The fusion's backward recomputes its per-view
terms from the inputs and the post-update volume; it must therefore run
before the next frame overwrites F and W.
"""
import torch

from . import ops


class SplatFn(torch.autograd.Function):
    """(depth, colour) -> (rgb, depth, alpha); colour = rgb_u8 / 255.

    ``colour`` is the float view of the 8-bit input that receives its
    gradient; the kernels read ``rgb_u8``, so ``colour`` must equal
    rgb_u8 / 255 (it is not read)."""

    @staticmethod
    def forward(ctx, depth, colour, rgb_u8, src, tgt, params):
        out = ops.splat_views(src, depth.detach(), rgb_u8, tgt, params, tape=True)
        ctx.save_for_backward(depth, rgb_u8, out["win_idx"], out["depth"], out["rgb"], out["tape"])
        ctx.cams = (ops.cameras(src), ops.camera(tgt), ops.splat_params(params))
        ctx.mark_non_differentiable(out["win_idx"])
        return out["rgb"], out["depth"], out["alpha"], out["win_idx"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, _g_win):
        depth, rgb_u8, win, od, orgb, tape = ctx.saved_tensors
        src, tgt, params = ctx.cams
        fwd = dict(win_idx=win, depth=od, rgb=orgb, tape=tape)

        def c(t):
            return None if t is None else t.contiguous()

        gd, gc = ops.splat_views_backward(src, depth.detach(), rgb_u8, tgt, params, fwd,
                                          c(g_rgb), c(g_depth), c(g_alpha))
        return gd, gc, None, None, None, None


class TsdfFn(torch.autograd.Function):
    """depth -> fused, extracted target depth (plus bin, F, W, not
    differentiable).  F_prev / W_prev (optional) carry the previous frame;
    F / W may alias them (in-place update)."""

    @staticmethod
    def forward(ctx, depth, src, tgt, params, F_prev, W_prev, F, W, mask):
        F, W, dep, b = ops.tsdf_integrate(src, depth.detach(), tgt, params, F_prev=F_prev,
                                          W_prev=W_prev, F=F, W=W, mask=mask, extract=True)
        ctx.save_for_backward(depth, F, W, b)
        ctx.cams = (ops.cameras(src), ops.camera(tgt), ops.tsdf_params(params))
        ctx.mark_non_differentiable(b, F, W)
        return dep, b, F, W

    @staticmethod
    def backward(ctx, g_dep, _gb, _gF, _gW):
        depth, F, W, b = ctx.saved_tensors
        src, tgt, params = ctx.cams
        if g_dep is None:
            return (None,) * 9
        g2 = ops.tsdf_extract_depth_backward(tgt, params, F, W, b, g_dep.contiguous())
        gd = ops.tsdf_integrate_backward(src, depth.detach(), tgt, params, F, W, b, g2)
        return gd, None, None, None, None, None, None, None, None


def splat(src, depth, rgb_u8, tgt, params, colour=None):
    """Differentiable splat.  Pass ``colour`` (float32, requires_grad, equal
    to rgb_u8 / 255) to receive colour gradients."""
    if colour is None:
        colour = torch.zeros(rgb_u8.shape, dtype=torch.float32, device=rgb_u8.device)
    return SplatFn.apply(depth, colour, rgb_u8, src, tgt, params)


def tsdf(src, depth, tgt, params, F_prev=None, W_prev=None, F=None, W=None, mask=None):
    """Differentiable fusion + extraction; returns (depth, bin, F, W)."""
    return TsdfFn.apply(depth, src, tgt, params, F_prev, W_prev, F, W, mask)
