"""Differentiable ray-tracer: images and SEDs as functions of the density.

Forward is ``mcrt_raytrace_image`` with the traced density passed as
``rho_rt``; backward is ``mcrt_raytrace_adjoint`` (the hand-written adjoint
of the formal solution of sect. 4, Eqs. 12-17, that recomputes the
transmittance in a second front-to-back sweep instead of storing it).
"""
from __future__ import annotations

import torch


class RaytraceImage(torch.autograd.Function):
    """rho [cells] (device, context precision) -> (images, sed)."""

    @staticmethod
    def forward(ctx_, rho, mctx, npx, npy):
        rho = rho.contiguous()
        img, sed = mctx.raytrace_device(npx, npy, rho_rt=rho)
        ctx_.save_for_backward(rho)
        ctx_.mctx, ctx_.npx, ctx_.npy = mctx, npx, npy
        return img, sed

    @staticmethod
    def backward(ctx_, g_img, g_sed):
        (rho,) = ctx_.saved_tensors
        m = ctx_.mctx
        dt = torch.float64 if m.fp64 else torch.float32
        gi = None if g_img is None else g_img.to(dt).contiguous()
        gs = None if g_sed is None else g_sed.to(torch.float64).contiguous()
        grad = m.raytrace_adjoint_device(ctx_.npx, ctx_.npy, w_img=gi, w_sed=gs, rho_rt=rho)
        return grad, None, None, None


def raytrace(rho, mctx, npx, npy):
    return RaytraceImage.apply(rho, mctx, npx, npy)
