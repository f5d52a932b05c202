"""torch.autograd wrappers: the forward calls the fused HIP step (saving the
limiter mask), the backward calls the hand-written adjoint kernels.

Tensors use the canonical contiguous layouts (k, j, i):
  u       (nk, nj+4, ni+4)  -- domain plus its 2-point halo
  data    (nk, nj, ni)
  w       (nk+1, nj, ni)    -- staggered levels
  coeff   a float, a 0-d tensor, or a per-point field (nk, nj, ni)
Outputs are the new interior values (nk, nj, ni).  Gradients of the step
flow to u (over its halo as well), data, w and a tensor coeff (scalar or
field); the step is differentiated almost everywhere, with the limiter
decisions of the forward pass held fixed (and d|t|/dt = 0 at t = 0 in the
diagonal of T).  `damping=True` selects the damping form of the diffusion.
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


def _opts(coeff, damping):
    """Options of the generalised diffusion: the damping form and, for a
    coefficient tensor with dimensions, the per-point field."""
    field = torch.is_tensor(coeff) and coeff.dim() == 3
    return api.Options(hdiff_form=api.HDIFF_DAMPING if damping else api.HDIFF_STATED,
                       coeff_field=_f(coeff, 0) if field else None), field


class StencilStep(torch.autograd.Function):
    """x = vadv(hdiff(u), data, w): one fused time step.  coeff may be a
    float, a 0-d tensor or a per-point field; gradients flow to u, data, w
    and a tensor coeff."""

    @staticmethod
    def forward(ctx, u, data, w, coeff, dt_dz: float, damping: bool = False):
        u, data, w = u.contiguous(), data.contiguous(), w.contiguous()
        ni, nj, nk = _dims(data)
        dom = (ni, nj, nk)
        if torch.is_tensor(coeff) and coeff.dim() == 3:
            coeff = coeff.contiguous()
        opts, field = _opts(coeff, damping)
        c = 0.0 if field else float(coeff)
        out = torch.empty_like(data)
        mask = torch.empty(max(api.stencil_mask_bytes(dom), 1), dtype=torch.uint8, device=u.device)
        api.stencil_step(_f(u, HALO), _f(data, 0), _f(w, 0), _f(out, 0), dom, c, dt_dz, mask=mask, opts=opts)
        ctx.params = ctx.needs_input_grad[2] or (torch.is_tensor(coeff) and ctx.needs_input_grad[3])
        # the parameter gradients need the step's input and output
        ctx.save_for_backward(w, mask, u if ctx.params else None, out if ctx.params else None,
                              coeff if field else None)
        ctx.coeff, ctx.dt_dz, ctx.dom, ctx.damping, ctx.field = c, dt_dz, dom, damping, field
        ctx.coeff_tensor = torch.is_tensor(coeff)
        return out

    @staticmethod
    def backward(ctx, xbar):
        w, mask, u, out, kap = ctx.saved_tensors
        ni, nj, nk = ctx.dom
        opts, _ = _opts(kap if ctx.field else ctx.coeff, ctx.damping)
        xbar = xbar.contiguous()
        ubar = torch.empty((nk, nj + 2 * HALO, ni + 2 * HALO), dtype=xbar.dtype, device=xbar.device)
        dbar = torch.empty_like(xbar)
        api.stencil_step_adjoint(_f(xbar, 0), _f(w, 0), mask, _f(ubar, HALO), _f(dbar, 0), ctx.dom, ctx.coeff,
                                 ctx.dt_dz, opts=opts)
        wbar = cbar = None
        if ctx.params:
            want_w = ctx.needs_input_grad[2]
            want_c = ctx.coeff_tensor and ctx.needs_input_grad[3]
            if want_c and ctx.field:
                kb = torch.empty_like(xbar)
                api.stencil_coeff_field_adjoint(_f(u, HALO), _f(dbar, 0), _f(kb, 0), ctx.dom, opts=opts)
                cbar = kb
            want_scalar = want_c and not ctx.field
            if want_w or want_scalar:
                wb = torch.empty_like(w) if want_w else None
                cb = torch.zeros(1, dtype=torch.float64, device=xbar.device) if want_scalar else None
                n = api.stencil_param_workspace_bytes(xbar.dtype, ctx.dom) if want_scalar else 0
                ws = torch.empty(n, dtype=torch.uint8, device=xbar.device) if n else None
                api.stencil_step_param_adjoint(_f(u, HALO), _f(w, 0), _f(out, 0), _f(dbar, 0),
                                               _f(wb, 0) if want_w else None, cb, ctx.dom, ctx.dt_dz, ws=ws,
                                               dtype=xbar.dtype, opts=opts)
                wbar = wb
                if want_scalar:
                    cbar = cb.reshape(()).to(xbar.dtype)
        return ubar, dbar, wbar, cbar, None, None


class HDiff(torch.autograd.Function):
    """out = hdiff(u) on the interior; coeff a float, a 0-d tensor or a
    per-point field, with gradients to u and a tensor coeff."""

    @staticmethod
    def forward(ctx, u, coeff, damping: bool = False):
        u = u.contiguous()
        nk, Nj, Ni = u.shape
        dom = (Ni - 2 * HALO, Nj - 2 * HALO, nk)
        if torch.is_tensor(coeff) and coeff.dim() == 3:
            coeff = coeff.contiguous()
        opts, field = _opts(coeff, damping)
        c = 0.0 if field else float(coeff)
        out = torch.empty((nk, dom[1], dom[0]), dtype=u.dtype, device=u.device)
        mask = torch.empty(max(api.stencil_mask_bytes(dom), 1), dtype=torch.uint8, device=u.device)
        api.stencil_hdiff(_f(u, HALO), _f(out, 0), dom, c, mask=mask, opts=opts)
        want_c = torch.is_tensor(coeff) and ctx.needs_input_grad[1]
        ctx.save_for_backward(mask, u if want_c else None, coeff if field else None)
        ctx.coeff, ctx.dom, ctx.damping, ctx.field, ctx.want_c = c, dom, damping, field, want_c
        return out

    @staticmethod
    def backward(ctx, obar):
        mask, u, kap = ctx.saved_tensors
        ni, nj, nk = ctx.dom
        opts, _ = _opts(kap if ctx.field else ctx.coeff, ctx.damping)
        obar = obar.contiguous()
        ubar = torch.empty((nk, nj + 2 * HALO, ni + 2 * HALO), dtype=obar.dtype, device=obar.device)
        api.stencil_hdiff_adjoint(_f(obar, 0), mask, _f(ubar, HALO), ctx.dom, ctx.coeff, opts=opts)
        cbar = None
        if ctx.want_c and ctx.field:
            kb = torch.empty_like(obar)
            api.stencil_coeff_field_adjoint(_f(u, HALO), _f(obar, 0), _f(kb, 0), ctx.dom, opts=opts)
            cbar = kb
        elif ctx.want_c:  # the scalar: -sum obar * D(u), the parameter adjoint with lambda = obar
            cb = torch.zeros(1, dtype=torch.float64, device=obar.device)
            n = api.stencil_param_workspace_bytes(obar.dtype, ctx.dom)
            ws = torch.empty(n, dtype=torch.uint8, device=obar.device) if n else None
            api.stencil_step_param_adjoint(_f(u, HALO), None, None, _f(obar, 0), None, cb, ctx.dom, 0.5, ws=ws,
                                           dtype=obar.dtype, opts=opts)
            cbar = cb.reshape(()).to(obar.dtype)
        return ubar, cbar, None


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


def step(u, data, w, coeff=0.025, dt_dz=0.5, damping=False):
    return StencilStep.apply(u, data, w, coeff, dt_dz, damping)


def hdiff(u, coeff=0.025, damping=False):
    return HDiff.apply(u, coeff, damping)


def vadv(u, data, w, dt_dz=0.5):
    return VAdv.apply(u, data, w, dt_dz)
