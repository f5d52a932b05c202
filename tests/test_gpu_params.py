"""GPU parity of the parameter gradients of a step (coeff and w) against
the oracle, end to end (forward step, step adjoint, parameter adjoint) and
for the parameter kernels alone (fed the GPU's own x and lambda), plus the
autograd wiring and an exact difference quotient in coeff through the GPU
forward step."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, autograd, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32, unpack_mask

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = [torch.float64, torch.float32]
IDS = ["f64", "f32"]
CASES = [(64, 64, 16), (67, 45, 7), (1, 1, 1), (33, 17, 137), (130, 3, 2), (5, 70, 1)]


def _ref(f, dtype):
    if dtype == torch.float32:
        return inputs.Fields(u=round_f32(f.u), w=round_f32(f.w), data=round_f32(f.data))
    return f


def _gpu_chain(f, dims, dtype):
    """Forward step (mask saved), step adjoint (lambda = data_bar), parameter
    adjoint; returns the device fields and outputs."""
    ni, nj, nk = dims
    u, data, w = dev_fields(f, dtype, DEV)
    x = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    o = api.Options()
    o.workspace = fields.workspace(api.OP_STEP, dtype, dims, o)
    api.stencil_step(u, data, w, x, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=o)
    ob = inputs.cotangent(ni, nj, nk)
    xb = fields.from_interior(ob, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    lam = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, lam, dims, inputs.COEFF, inputs.DT_DZ)
    wb = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, kextra=1, fill=123.0)
    cb = torch.full((1,), 123.0, dtype=torch.float64, device=DEV)
    n = api.stencil_param_workspace_bytes(dtype, dims)
    ws = torch.empty(n, dtype=torch.uint8, device=DEV) if n else None
    api.stencil_step_param_adjoint(u, w, x, lam, wb, cb, dims, inputs.DT_DZ, ws=ws)
    torch.cuda.synchronize()
    return dict(u=u, w=w, x=x, lam=lam, wb=wb, cb=cb, mask=mask, ob=ob)


def _coeff_scale(u, lam, mx, my):
    """sum |lam * D(u)|: the condition scale of the coeff gradient's sum."""
    return float(np.sum(np.abs(lam * orc.hdiff_divergence(u, mx, my))))


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("dims", CASES, ids=lambda d: "x".join(map(str, d)))
def test_param_gradients_vs_oracle(dims, dtype):
    ni, nj, nk = dims
    print(f"param adjoint {dims} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=401)
    r = _ref(f, dtype)
    g = _gpu_chain(f, dims, dtype)
    coeff = c_scalar(inputs.COEFF, dtype)
    nxt, mx, my = orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=(dtype == torch.float32))
    ob = round_f32(g["ob"]) if dtype == torch.float32 else g["ob"]
    lam = orc.vadv_adjoint(ob, r.w, inputs.DT_DZ)
    wbar = orc.w_grad(r.w, nxt[:, 2:-2, 2:-2], lam, inputs.DT_DZ)
    cbar = orc.coeff_grad(r.u, lam, mx, my)
    # the masks the GPU used are the oracle's (bit for bit)
    gx, gy = unpack_mask(g["mask"], ni, nj, nk)
    assert np.array_equal(gx, mx) and np.array_equal(gy, my)
    got_w = host(fields.interior(g["wb"], ni, nj, nk + 1))
    assert rel_err(got_w, wbar) <= TOL[dtype], dims
    scale = max(_coeff_scale(r.u, lam, mx, my), 1e-300)
    assert abs(float(g["cb"].item()) - cbar) <= TOL[dtype] * scale, (dims, g["cb"].item(), cbar)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
def test_param_kernels_alone(dtype):
    """The parameter kernels fed the GPU's own x and lambda: the oracle on the
    same (upcast) values isolates the kernels' arithmetic."""
    dims = (75, 41, 23)
    ni, nj, nk = dims
    f = inputs.fields_sized(ni, nj, nk, seed=402)
    r = _ref(f, dtype)
    g = _gpu_chain(f, dims, dtype)
    x = host(fields.interior(g["x"], ni, nj, nk))
    lam = host(fields.interior(g["lam"], ni, nj, nk))
    mx, my = unpack_mask(g["mask"], ni, nj, nk)
    wbar = orc.w_grad(r.w, x, lam, inputs.DT_DZ)
    cbar = orc.coeff_grad(r.u, lam, mx, my)
    tol = 1e-14 if dtype == torch.float64 else 1e-5
    assert rel_err(host(fields.interior(g["wb"], ni, nj, nk + 1)), wbar) <= tol
    assert abs(float(g["cb"].item()) - cbar) <= tol * _coeff_scale(r.u, lam, mx, my)


def test_param_gradients_full_size():
    """512 x 512 x 80 FP64, the fused-step benchmark size."""
    dims = (512, 512, 80)
    ni, nj, nk = dims
    f = inputs.fields_for(inputs.STEP_512)
    g = _gpu_chain(f, dims, torch.float64)
    nxt, mx, my = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    lam = orc.vadv_adjoint(g["ob"], f.w, inputs.DT_DZ)
    wbar = orc.w_grad(f.w, nxt[:, 2:-2, 2:-2], lam, inputs.DT_DZ)
    cbar = orc.coeff_grad(f.u, lam, mx, my)
    assert rel_err(host(fields.interior(g["wb"], ni, nj, nk + 1)), wbar) <= 1e-12
    assert abs(float(g["cb"].item()) - cbar) <= 1e-12 * _coeff_scale(f.u, lam, mx, my)


def test_coeff_gradient_exact_quotient_on_gpu():
    """<ob, step> is affine in coeff (the limiter does not depend on it): the
    GPU forward's central quotient equals the GPU gradient to rounding."""
    dims = (96, 80, 40)
    ni, nj, nk = dims
    f = inputs.fields_sized(ni, nj, nk, seed=403)
    g = _gpu_chain(f, dims, torch.float64)
    u, data, w = dev_fields(f, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0)

    def loss(c):
        api.stencil_step(u, data, w, out, dims, c, inputs.DT_DZ)
        torch.cuda.synchronize()
        return math.fsum((host(fields.interior(out, ni, nj, nk)) * g["ob"]).ravel())

    h = 0.01
    fd = (loss(inputs.COEFF + h) - loss(inputs.COEFF - h)) / (2 * h)
    cb = float(g["cb"].item())
    assert abs(fd - cb) <= 1e-9 * max(1.0, abs(cb)), (fd, cb)


def test_autograd_parameter_gradients():
    """StencilStep with w and a tensor coeff requiring grad: the gradients are
    the parameter adjoint's, and u / data keep theirs."""
    ni, nj, nk = 40, 24, 12
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=404)
    dt = torch.float64
    u = torch.tensor(f.u, dtype=dt, device=DEV, requires_grad=True)
    data = torch.tensor(f.data, dtype=dt, device=DEV, requires_grad=True)
    w = torch.tensor(f.w, dtype=dt, device=DEV, requires_grad=True)
    c = torch.tensor(inputs.COEFF, dtype=dt, device=DEV, requires_grad=True)
    ob = torch.tensor(inputs.cotangent(ni, nj, nk), dtype=dt, device=DEV)
    x = autograd.step(u, data, w, c, inputs.DT_DZ)
    (x * ob).sum().backward()
    g = _gpu_chain(f, dims, dt)
    assert torch.equal(w.grad, fields.interior(g["wb"], ni, nj, nk + 1))
    assert torch.equal(data.grad, fields.interior(g["lam"], ni, nj, nk))
    assert abs(c.grad.item() - g["cb"].item()) <= 1e-12 * max(1.0, abs(g["cb"].item()))
    assert u.grad.shape == u.shape
