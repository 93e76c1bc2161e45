"""Differentiable form of the forward model: w -> p = P f(f0, xbar + U w).

``project`` is a ``torch.autograd.Function`` whose forward runs the fused
DVF + warp kernel and the cone-beam projection, and whose hand-written
backward is exactly the adjoint path of the solve: the back-projection
``drr_adjoint`` of the incoming image gradient followed by the Jacobian chain
``grad_w`` (Appendix: dJ/dw = 2 U^T (df/dx) P^T r; here without the factor 2,
since the incoming gradient already is dL/dp).

The backward needs f0, xbar, U and w -- the Jacobian of Eqs. A.4-A.8 reads the
reference image's neighbours at the pulled-back positions -- so the warped
volume is never stored: it is recomputed only if another forward is asked
for.  ``store_warp=True`` keeps it anyway (for callers that want f), which
costs one volume of HBM and changes nothing in the gradient.

w is a small host tensor (float64, K <= 8); p and its gradient live on the
GPU in the volume's dtype.  Marshalling only: every step runs in libpcasolve.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding as B


class _ProjectWarp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, vol, proj, rays, f0, mean, U, store_warp: bool):
        w_host = w.detach().to("cpu", torch.float64).contiguous()
        f = B.warp_pca(vol, f0, mean, U, w_host)
        p = B.drr_forward(vol, proj, rays, f)
        ctx.vol, ctx.proj = vol, proj
        # saved through autograd so that an in-place change of the ray
        # table or the model between forward and backward raises instead of
        # silently mixing two geometries
        ctx.save_for_backward(rays, f0, mean, U)
        ctx.w_host = w_host
        ctx.w_device, ctx.w_dtype = w.device, w.dtype
        ctx.f = f if store_warp else None
        return p

    @staticmethod
    def backward(ctx, grad_p):
        g = None
        if ctx.needs_input_grad[0]:
            rays, f0, mean, U = ctx.saved_tensors
            gp = grad_p.contiguous().to(f0.dtype)
            bp = B.drr_adjoint(ctx.vol, ctx.proj, rays, gp)
            g2 = B.grad_w(ctx.vol, f0, mean, U, ctx.w_host, bp)
            # grad_w returns 2 U^T (df/dx) bp (dJ/dw of Eq. 2, where
            # dJ/dp = 2 r); halving it is exact in binary floating point
            g = (0.5 * g2).to(device=ctx.w_device, dtype=ctx.w_dtype)
        return g, None, None, None, None, None, None, None


def project(w, vol, proj, rays, f0, mean, U, store_warp: bool = False):
    """p = P f(f0, mean + U w), differentiable in w."""
    return _ProjectWarp.apply(w, vol, proj, rays, f0, mean, U, store_warp)


class PCAProjector(torch.nn.Module):
    """Holds the resident reference image, motion model and ray table of one
    projection geometry; ``forward(w)`` returns the projection image."""

    def __init__(self, vol, proj, f0, mean: Optional[torch.Tensor], U, store_warp: bool = False):
        super().__init__()
        self.vol, self.proj = vol, proj
        self.f0, self.mean, self.U = f0, mean, U
        self.store_warp = store_warp
        self.rays = B.ray_table(vol, proj, f0.dtype)

    def set_projection(self, proj):
        """Switch to another geometry.  A fresh ray table is built, so graphs
        recorded at the previous angle keep theirs for their backward."""
        self.proj = proj
        self.rays = B.ray_table(self.vol, proj, self.f0.dtype)

    def forward(self, w):
        return project(w, self.vol, self.proj, self.rays, self.f0, self.mean, self.U,
                       self.store_warp)
