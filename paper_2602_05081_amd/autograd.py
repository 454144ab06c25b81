"""torch.autograd.Function over the optical-depth kernels.

Forward calls gf_optical_depth (tau and T = exp(-tau)); backward calls
gf_optical_depth_backward with dL/dtau and dL/dT, which re-traverses the
LBVH and recomputes every segment (no stored paths).  The scene is rebuilt
from the parameter tensor on each forward call, so gradients are with respect
to the caller's 15-float records.
"""
from __future__ import annotations

import torch

from . import _lib


class GaborOpticalDepth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, rays, rho, mask_cells=_lib.FULL_CELLS, image_width=0, trunc_r=3.0):
        scene = _lib.Scene(params.detach().contiguous(), rho, trunc_r)
        tau, T = _lib.gf_optical_depth(scene, rays, _lib.make_mask(mask_cells), image_width)
        ctx.scene = scene
        ctx.mask_cells = mask_cells
        ctx.image_width = image_width
        ctx.save_for_backward(rays, T)
        return tau, T

    @staticmethod
    def backward(ctx, g_tau, g_T):
        rays, T = ctx.saved_tensors
        if g_tau is None:
            g_tau = torch.zeros_like(T)
        g_tau = g_tau.contiguous().float()
        gT = None if g_T is None else g_T.contiguous().float()
        grad = _lib.gf_optical_depth_backward(ctx.scene, rays, g_tau, _lib.make_mask(ctx.mask_cells), gT,
                                              None if gT is None else T, ctx.image_width)
        ctx.scene.close()
        return grad, None, None, None, None, None


def optical_depth(params, rays, rho, mask_cells=_lib.FULL_CELLS, image_width=0, trunc_r=3.0):
    """(tau, T) per ray, differentiable with respect to params (n x 15)."""
    return GaborOpticalDepth.apply(params, rays, rho, mask_cells, image_width, trunc_r)
