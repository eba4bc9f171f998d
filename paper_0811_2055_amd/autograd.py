"""Differentiable splat: a torch.autograd.Function over splat_render and its
hand-written adjoint (splat_render_backward), both HIP kernels in liblod.so.

For the Gaussian blob the derivative of the truncation indicator is taken as
zero (the derivative almost everywhere), so gradients flow only through the
Gaussian weights and the projection; the radial cubic blob has no edge.
"""
from __future__ import annotations

import torch

from . import lib


class SplatRender(torch.autograd.Function):
    """image = splat(x, y, z, m) for one camera; gradients w.r.t. x, y, z, m."""

    @staticmethod
    def forward(ctx, x, y, z, m, cam, sigma, radius_sigmas, workspace, blob=None):
        for t in (x, y, z, m):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise TypeError("SplatRender takes float32 device tensors")
        x, y, z, m = (t.contiguous() for t in (x, y, z, m))
        img = lib.splat(x, y, z, m, cam, sigma, radius_sigmas, workspace=workspace, blob=blob)
        ctx.save_for_backward(x, y, z, m)
        ctx.cam, ctx.sigma, ctx.radius, ctx.blob = cam, sigma, radius_sigmas, blob
        return img

    @staticmethod
    def backward(ctx, grad_img):
        x, y, z, m = ctx.saved_tensors
        gm, gx, gy, gz = lib.splat_backward(x, y, z, m, grad_img.contiguous(), ctx.cam, ctx.sigma, ctx.radius,
                                            blob=ctx.blob)
        return gx, gy, gz, gm, None, None, None, None, None


def splat_render(x, y, z, m, cam, sigma: float = 1.0, radius_sigmas: float = 3.0, workspace=None, blob=None):
    return SplatRender.apply(x, y, z, m, cam, sigma, radius_sigmas, workspace, blob)
