"""torch.autograd wrappers: the forward calls the fused HIP step (saving the
limiter mask), the backward calls the hand-written adjoint kernels.

Tensors use the canonical contiguous layouts (k, j, i):
  u       (nk, nj+4, ni+4)  -- domain plus its 2-point halo
  data    (nk, nj, ni)
  w       (nk+1, nj, ni)    -- staggered levels
Outputs are the new interior values (nk, nj, ni).  Gradients of the step
flow to u (over its halo as well), data, w and a tensor coeff; the step is
differentiated almost everywhere, with the limiter decisions of the forward
pass held fixed (and d|t|/dt = 0 at t = 0 in the diagonal of T).
"""
from __future__ import annotations

import torch

from . import api

HALO = 2


def _f(t: torch.Tensor, halo: int) -> api.Field:
    return api.Field(t, (halo, halo, 0))


def _dims(data: torch.Tensor):
    nk, nj, ni = data.shape
    return ni, nj, nk


class StencilStep(torch.autograd.Function):
    """x = vadv(hdiff(u), data, w): one fused time step.  coeff may be a
    float or a 0-d tensor; gradients flow to u, data, w and a tensor coeff."""

    @staticmethod
    def forward(ctx, u, data, w, coeff, dt_dz: float):
        u, data, w = u.contiguous(), data.contiguous(), w.contiguous()
        ni, nj, nk = _dims(data)
        dom = (ni, nj, nk)
        c = float(coeff)
        out = torch.empty_like(data)
        mask = torch.empty(max(api.stencil_mask_bytes(dom), 1), dtype=torch.uint8, device=u.device)
        api.stencil_step(_f(u, HALO), _f(data, 0), _f(w, 0), _f(out, 0), dom, c, dt_dz, mask=mask)
        ctx.params = ctx.needs_input_grad[2] or (torch.is_tensor(coeff) and ctx.needs_input_grad[3])
        # the parameter gradients need the step's input and output
        ctx.save_for_backward(w, mask, u if ctx.params else None, out if ctx.params else None)
        ctx.coeff, ctx.dt_dz, ctx.dom = c, dt_dz, dom
        ctx.coeff_tensor = torch.is_tensor(coeff)
        return out

    @staticmethod
    def backward(ctx, xbar):
        w, mask, u, out = ctx.saved_tensors
        ni, nj, nk = ctx.dom
        xbar = xbar.contiguous()
        ubar = torch.empty((nk, nj + 2 * HALO, ni + 2 * HALO), dtype=xbar.dtype, device=xbar.device)
        dbar = torch.empty_like(xbar)
        api.stencil_step_adjoint(_f(xbar, 0), _f(w, 0), mask, _f(ubar, HALO), _f(dbar, 0), ctx.dom, ctx.coeff,
                                 ctx.dt_dz)
        wbar = cbar = None
        if ctx.params:
            want_w = ctx.needs_input_grad[2]
            want_c = ctx.coeff_tensor and ctx.needs_input_grad[3]
            wb = torch.empty_like(w) if want_w else None
            cb = torch.zeros(1, dtype=torch.float64, device=xbar.device) if want_c else None
            n = api.stencil_param_workspace_bytes(xbar.dtype, ctx.dom) if want_c else 0
            ws = torch.empty(n, dtype=torch.uint8, device=xbar.device) if n else None
            api.stencil_step_param_adjoint(_f(u, HALO), _f(w, 0), _f(out, 0), _f(dbar, 0),
                                           _f(wb, 0) if want_w else None, cb, ctx.dom, ctx.dt_dz, ws=ws,
                                           dtype=xbar.dtype)
            wbar = wb
            cbar = cb.reshape(()).to(xbar.dtype) if want_c else None
        return ubar, dbar, wbar, cbar, None


class HDiff(torch.autograd.Function):
    """out = hdiff(u) on the interior."""

    @staticmethod
    def forward(ctx, u, coeff: float):
        u = u.contiguous()
        nk, Nj, Ni = u.shape
        dom = (Ni - 2 * HALO, Nj - 2 * HALO, nk)
        out = torch.empty((nk, dom[1], dom[0]), dtype=u.dtype, device=u.device)
        mask = torch.empty(max(api.stencil_mask_bytes(dom), 1), dtype=torch.uint8, device=u.device)
        api.stencil_hdiff(_f(u, HALO), _f(out, 0), dom, coeff, mask=mask)
        ctx.save_for_backward(mask)
        ctx.coeff, ctx.dom = coeff, dom
        return out

    @staticmethod
    def backward(ctx, obar):
        (mask,) = ctx.saved_tensors
        ni, nj, nk = ctx.dom
        obar = obar.contiguous()
        ubar = torch.empty((nk, nj + 2 * HALO, ni + 2 * HALO), dtype=obar.dtype, device=obar.device)
        api.stencil_hdiff_adjoint(_f(obar, 0), mask, _f(ubar, HALO), ctx.dom, ctx.coeff)
        return ubar, None


class VAdv(torch.autograd.Function):
    """x = T(w)^{-1} (u + data) per column."""

    @staticmethod
    def forward(ctx, u, data, w, dt_dz: float):
        u, data, w = u.contiguous(), data.contiguous(), w.contiguous()
        dom = _dims(data)
        out = torch.empty_like(data)
        api.stencil_vadv(_f(u, 0), _f(data, 0), _f(w, 0), _f(out, 0), dom, dt_dz)
        ctx.save_for_backward(w)
        ctx.dt_dz, ctx.dom = dt_dz, dom
        return out

    @staticmethod
    def backward(ctx, xbar):
        (w,) = ctx.saved_tensors
        xbar = xbar.contiguous()
        lam = torch.empty_like(xbar)
        api.stencil_vadv_adjoint(_f(xbar, 0), _f(w, 0), _f(lam, 0), ctx.dom, ctx.dt_dz)
        return lam, lam, None, None


def step(u, data, w, coeff=0.025, dt_dz=0.5):
    return StencilStep.apply(u, data, w, coeff, dt_dz)


def hdiff(u, coeff=0.025):
    return HDiff.apply(u, coeff)


def vadv(u, data, w, dt_dz=0.5):
    return VAdv.apply(u, data, w, dt_dz)
