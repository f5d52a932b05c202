"""Fields whose levels span more than 2 GiB.

Every kernel addresses a level through a buffer descriptor (64-bit level
base) plus a 32-bit byte offset per lane, so a level may be up to about
4 GiB.  Here a level of every field holds more than 2^31 bytes, so the
offsets of the far rows have their top bit set.  The step, the diffusion
alone and the step adjoint run on the whole domain in their default launch
configuration; outputs are then checked at sampled windows against the
oracle run on the window with its neighbourhood (the step's output at a
point depends on u within two points and on its own column; the adjoint's
u_bar at a point on x_bar within two points), near the first and the last
rows and columns and in the middle.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, host, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda"
W8 = 8  # window width of the checked outputs


def _windows(ni, nj):
    e = W8
    return [(0, 0), (ni - e, nj - e), (ni // 2 + 3, nj - e), (5, nj - e - 3), (ni - e, 0),
            (ni - 13, nj // 2 + 101)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_levels_beyond_2gib(dtype):
    es = 8 if dtype == torch.float64 else 4
    n = 16400 if es == 8 else 23200
    ni, nj, nk = n, n, 3
    dims = (ni, nj, nk)
    f32 = dtype == torch.float32
    print(f"levels beyond 2 GiB: {dims} {dtype}", flush=True)
    u = fields.alloc(ni, nj, nk, dtype, DEV)
    data = fields.alloc(ni, nj, nk, dtype, DEV, halo=0)
    w = fields.alloc(ni, nj, nk + 1, dtype, DEV, halo=0)
    for fl in (u, data, w):
        assert fl.tensor.stride(0) * es > 2**31
    U = fields.padded(u, ni, nj, nk)
    D = fields.interior(data, ni, nj, nk)
    Wf = fields.interior(w, ni, nj, nk + 1)
    inputs.fill_device([U, Wf, D], inputs.FIELD_RANGES, inputs.LARGE_CHILD)
    coeff = c_scalar(inputs.COEFF, dtype)

    # forward step (saving the limiter mask) and the diffusion alone
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask)
    hd = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    api.stencil_hdiff(u, hd, dims, inputs.COEFF)
    torch.cuda.synchronize()
    O = fields.interior(out, ni, nj, nk)
    H = fields.interior(hd, ni, nj, nk)
    for i0, j0 in _windows(ni, nj):
        uw = host(U[:, j0:j0 + W8 + 4, i0:i0 + W8 + 4])
        dw = host(D[:, j0:j0 + W8, i0:i0 + W8])
        ww = host(Wf[:, j0:j0 + W8, i0:i0 + W8])
        ref, _, _ = orc.step(uw, dw, ww, coeff, inputs.DT_DZ, decide_f32=f32)
        e = rel_err(host(O[:, j0:j0 + W8, i0:i0 + W8]), ref[:, 2:-2, 2:-2])
        assert e <= TOL[dtype], f"step window ({i0}, {j0}): {e:.2e}"
        href, _, _ = orc.hdiff(uw, coeff, decide_f32=f32)
        e = rel_err(host(H[:, j0:j0 + W8, i0:i0 + W8]), href[:, 2:-2, 2:-2])
        assert e <= TOL[dtype], f"hdiff window ({i0}, {j0}): {e:.2e}"
    del out, hd, O, H, data, D
    torch.cuda.empty_cache()

    # step adjoint with the forward's mask
    xb = fields.alloc(ni, nj, nk, dtype, DEV, halo=0)
    XB = fields.interior(xb, ni, nj, nk)
    inputs.fill_device([XB], [inputs.COTANGENT_RANGE], inputs.LARGE_CHILD + 1)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    db = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ)
    torch.cuda.synchronize()
    UB = fields.interior(ub, ni, nj, nk)
    DB = fields.interior(db, ni, nj, nk)
    for i0, j0 in _windows(ni, nj):
        # the window grown by two points, clipped to the domain: every x_bar
        # that reaches the checked points lies inside it
        a0, a1 = max(i0 - 2, 0), min(i0 + W8 + 2, ni)
        b0, b1 = max(j0 - 2, 0), min(j0 + W8 + 2, nj)
        uw = host(U[:, b0:b1 + 4, a0:a1 + 4])
        mx, my = orc.hdiff_masks(uw, decide_f32=f32)
        ubr, dbr = orc.step_adjoint(host(XB[:, b0:b1, a0:a1]), host(Wf[:, b0:b1, a0:a1]), mx, my, coeff,
                                    inputs.DT_DZ)
        ci, cj = i0 - a0 + 2, j0 - b0 + 2  # the checked points in the window's padded layout
        e = rel_err(host(UB[:, j0:j0 + W8, i0:i0 + W8]), ubr[:, cj:cj + W8, ci:ci + W8])
        assert e <= TOL[dtype], f"u_bar window ({i0}, {j0}): {e:.2e}"
        e = rel_err(host(DB[:, j0:j0 + W8, i0:i0 + W8]), dbr[:, cj - 2:cj - 2 + W8, ci - 2:ci - 2 + W8])
        assert e <= TOL[dtype], f"data_bar window ({i0}, {j0}): {e:.2e}"
    del u, w, U, Wf, xb, XB, ub, db, UB, DB, mask
    torch.cuda.empty_cache()
