"""GPU parity of the adjoint kernels: against the oracle's transposed
formulas, a dot-product test against the oracle's tangent-linear map, and
central finite differences of the GPU forward step."""
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


def _forward(f, dtype, dims):
    u, data, w = dev_fields(f, dtype, DEV)
    ni, nj, nk = dims
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    o = api.Options()
    o.workspace = fields.workspace(api.OP_STEP, dtype, dims, o)  # columns beyond the fused classes
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=o)
    return u, data, w, out, mask


def _ref(f, dtype):
    if dtype == torch.float32:
        return inputs.Fields(u=round_f32(f.u), w=round_f32(f.w), data=round_f32(f.data))
    return f


ADJ_CASES = [(64, 64, 16), (67, 45, 7), (1, 1, 1), (33, 17, 137), (20, 20, 161), (3, 70, 97)]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("with_dbar", [True, False], ids=["dbar", "ws"])
@pytest.mark.parametrize("impl", [api.IMPL_AUTO, api.IMPL_PLAIN], ids=["auto", "plain"])
@pytest.mark.parametrize("dims", ADJ_CASES, ids=lambda d: "x".join(map(str, d)))
def test_step_adjoint(dims, impl, with_dbar, dtype):
    ni, nj, nk = dims
    print(f"step adjoint {dims} impl={impl} dbar={with_dbar} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=201)
    r = _ref(f, dtype)
    u, data, w, out, mask = _forward(f, dtype, dims)
    ob = inputs.cotangent(ni, nj, nk)
    obr = round_f32(ob) if dtype == torch.float32 else ob
    xb = fields.from_interior(ob, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=123.0)
    db = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0) if with_dbar else None
    o = api.Options(impl=impl)
    # without data_bar lambda lives in the workspace (plus the plain factors)
    op = api.OP_VADV_ADJOINT if with_dbar else api.OP_STEP_ADJOINT
    n = api.stencil_workspace_bytes(op, dtype, dims, o)
    if n:
        o.workspace = torch.empty(n, dtype=torch.uint8, device=DEV)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ, opts=o)
    torch.cuda.synchronize()
    coeff = c_scalar(inputs.COEFF, dtype)
    _, mx, my = orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=(dtype == torch.float32))
    ubr, dbr = orc.step_adjoint(obr, r.w, mx, my, coeff, inputs.DT_DZ)
    # every padded point is overwritten (the never-read corners with 0)
    assert rel_err(host(fields.padded(ub, ni, nj, nk)), ubr) <= TOL[dtype]
    if with_dbar:
        assert rel_err(host(fields.interior(db, ni, nj, nk)), dbr) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("tile", [64, 32, 16])
def test_hdiff_adjoint(tile, dtype):
    ni, nj, nk = 75, 41, 6
    f = inputs.fields_sized(ni, nj, nk, seed=202)
    r = _ref(f, dtype)
    u = fields.from_padded(f.u, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor((ni, nj, nk), DEV)
    api.stencil_hdiff(u, out, (ni, nj, nk), inputs.COEFF, mask=mask)
    lam = inputs.cotangent(ni, nj, nk)
    lamr = round_f32(lam) if dtype == torch.float32 else lam
    lb = fields.from_interior(lam, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=9.0)
    api.stencil_hdiff_adjoint(lb, mask, ub, (ni, nj, nk), inputs.COEFF,
                              opts=api.Options(tile_i=tile, tile_j=256 // tile))
    torch.cuda.synchronize()
    coeff = c_scalar(inputs.COEFF, dtype)
    mx, my = orc.hdiff_masks(r.u, decide_f32=(dtype == torch.float32))
    ubr = orc.hdiff_adjoint(lamr, mx, my, coeff)
    assert rel_err(host(fields.padded(ub, ni, nj, nk)), ubr) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("nk", [1, 2, 16, 80, 96, 97, 137, 160, 161])
def test_vadv_adjoint(nk, dtype):
    ni, nj = 70, 5
    f = inputs.fields_sized(ni, nj, nk, seed=203)
    wr = round_f32(f.w) if dtype == torch.float32 else f.w
    xb = inputs.cotangent(ni, nj, nk)
    xbr = round_f32(xb) if dtype == torch.float32 else xb
    x = fields.from_interior(xb, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    lam = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    o = api.Options()
    n = api.stencil_workspace_bytes(api.OP_VADV_ADJOINT, dtype, (ni, nj, nk), o)
    if n:
        o.workspace = torch.empty(n, dtype=torch.uint8, device=DEV)
    api.stencil_vadv_adjoint(x, w, lam, (ni, nj, nk), inputs.DT_DZ, opts=o)
    torch.cuda.synchronize()
    ref = orc.vadv_adjoint(xbr, wr, inputs.DT_DZ)
    assert rel_err(host(fields.interior(lam, ni, nj, nk)), ref) <= TOL[dtype]


def test_adjoint_full_size_and_dot_test():
    """The step-adjoint workload (256x256x80, FP64): oracle parity, and the
    dot test <J v, w> = <v, J^T w> with J v from the oracle's tangent."""
    wl = inputs.ADJ_256
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    f = inputs.fields_for(wl)
    u, data, w, out, mask = _forward(f, torch.float64, dims)
    ob = inputs.cotangent(ni, nj, nk)
    xb = fields.from_interior(ob, torch.float64, DEV)
    ub = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    db = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ)
    _, mx, my = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    ubr, dbr = orc.step_adjoint(ob, f.w, mx, my, inputs.COEFF, inputs.DT_DZ)
    gub = host(fields.padded(ub, ni, nj, nk))
    assert rel_err(gub, ubr) <= 1e-12
    assert rel_err(host(fields.interior(db, ni, nj, nk)), dbr) <= 1e-12
    v, wv = inputs.dot_vectors(ni, nj, nk)
    Jv = orc.step_tangent(v, f.w, mx, my, inputs.COEFF, inputs.DT_DZ)
    xw = fields.from_interior(wv, torch.float64, DEV)
    api.stencil_step_adjoint(xw, w, mask, ub, None, dims, inputs.COEFF, inputs.DT_DZ,
                             opts=api.Options(workspace=fields.workspace(api.OP_STEP_ADJOINT, torch.float64, dims)))
    JTw = host(fields.padded(ub, ni, nj, nk))
    lhs = math.fsum((Jv * wv).ravel())
    rhs = math.fsum((v * JTw).ravel())
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) <= 1e-10


def test_adjoint_full_size_f32_and_dot_test():
    """The step-adjoint workload (256x256x80) in FP32.  The forward's binary32
    limiter decisions equal the oracle's binary32 decisions bit for bit; u_bar
    and data_bar match the FP64 oracle fed the binary32-rounded w and
    cotangent at 2e-5; and the dot test <J v, w> = <v, J^T w>, with J v from
    the oracle's tangent and J^T w from the GPU in binary32, agrees to 1e-5
    relative: each of the 5.4 M components of J^T w carries a few binary32
    roundings (about 1e-7 relative) whose random signs largely cancel in the
    sum, so 1e-5 leaves a margin of about 100."""
    wl = inputs.ADJ_256
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    f = inputs.fields_for(wl)
    r = _ref(f, torch.float32)
    u, data, w, out, mask = _forward(f, torch.float32, dims)
    coeff = c_scalar(inputs.COEFF, torch.float32)
    _, mx, my = orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=True)
    gmx, gmy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gmx, mx) and np.array_equal(gmy, my)
    ob = inputs.cotangent(ni, nj, nk)
    xb = fields.from_interior(ob, torch.float32, DEV)
    ub = fields.alloc(ni, nj, nk, torch.float32, DEV, fill=0.0)
    db = fields.alloc(ni, nj, nk, torch.float32, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ)
    ubr, dbr = orc.step_adjoint(round_f32(ob), r.w, mx, my, coeff, inputs.DT_DZ)
    e_u = rel_err(host(fields.padded(ub, ni, nj, nk)), ubr)
    e_d = rel_err(host(fields.interior(db, ni, nj, nk)), dbr)
    v, wv = inputs.dot_vectors(ni, nj, nk)
    wv32 = round_f32(wv)
    Jv = orc.step_tangent(v, r.w, mx, my, coeff, inputs.DT_DZ)
    xw = fields.from_interior(wv32, torch.float32, DEV)
    api.stencil_step_adjoint(xw, w, mask, ub, None, dims, inputs.COEFF, inputs.DT_DZ,
                             opts=api.Options(workspace=fields.workspace(api.OP_STEP_ADJOINT, torch.float32, dims)))
    JTw = host(fields.padded(ub, ni, nj, nk))
    lhs = math.fsum((Jv * wv32).ravel())
    rhs = math.fsum((v * JTw).ravel())
    e_dot = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    print(f"FP32 adjoint 256x256x80: u_bar {e_u:.2e}, data_bar {e_d:.2e}, dot test {e_dot:.2e}", flush=True)
    assert e_u <= 2e-5 and e_d <= 2e-5
    assert e_dot <= 1e-5


def test_central_finite_differences():
    """64 seeded points of the padded u, h = 1e-6, FP64: the GPU adjoint
    against central differences of the GPU forward step, evaluated on the
    columns a point can influence (the radius-2 diamond, every level)."""
    wl = inputs.ADJ_256
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    f = inputs.fields_for(wl)
    u, data, w, out, mask = _forward(f, torch.float64, dims)
    ob = inputs.cotangent(ni, nj, nk)
    xb = fields.from_interior(ob, torch.float64, DEV)
    ub = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    db = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ)
    gub = host(fields.padded(ub, ni, nj, nk))
    h = 1e-6
    Nj, Ni = nj + 4, ni + 4
    up = fields.from_padded(f.u, torch.float64, DEV)
    outp = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    outm = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    mp = fields.mask_tensor(dims, DEV)
    mm = fields.mask_tensor(dims, DEV)
    checked = 0
    for p in inputs.fd_points(ni, nj, nk, 64):
        k, jp, ip = int(p // (Nj * Ni)), int((p // Ni) % Nj), int(p % Ni)
        view = fields.padded(up, ni, nj, nk)
        base = float(f.u[k, jp, ip])
        view[k, jp, ip] = base + h
        api.stencil_step(up, data, w, outp, dims, inputs.COEFF, inputs.DT_DZ, mask=mp)
        view[k, jp, ip] = base - h
        api.stencil_step(up, data, w, outm, dims, inputs.COEFF, inputs.DT_DZ, mask=mm)
        view[k, jp, ip] = base
        if not (torch.equal(mp, mask) and torch.equal(mm, mask)):
            continue  # a limiter kink within h: the a.e. derivative does not apply
        i, j = ip - 2, jp - 2
        i0, i1, j0, j1 = max(i - 2, 0), min(i + 3, ni), max(j - 2, 0), min(j + 3, nj)
        if i0 >= i1 or j0 >= j1:
            fd = 0.0
        else:
            a = host(fields.interior(outp, ni, nj, nk)[:, j0:j1, i0:i1])
            b = host(fields.interior(outm, ni, nj, nk)[:, j0:j1, i0:i1])
            fd = math.fsum(((a - b) * ob[:, j0:j1, i0:i1]).ravel()) / (2 * h)
        g = gub[k, jp, ip]
        assert abs(fd - g) <= 1e-7 * max(1.0, abs(g)), (p, fd, g)
        checked += 1
    assert checked >= 56


def test_autograd_wiring():
    ni, nj, nk = 40, 24, 12
    f = inputs.fields_sized(ni, nj, nk, seed=204)
    u = torch.tensor(f.u, device=DEV, requires_grad=True)
    data = torch.tensor(f.data, device=DEV, requires_grad=True)
    w = torch.tensor(f.w, device=DEV)
    x = autograd.step(u, data, w, inputs.COEFF, inputs.DT_DZ)
    ob = torch.tensor(inputs.cotangent(ni, nj, nk), device=DEV)
    (x * ob).sum().backward()
    ref, mx, my = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    assert rel_err(host(x), ref[:, 2:-2, 2:-2]) <= 1e-12
    ubr, dbr = orc.step_adjoint(host(ob), f.w, mx, my, inputs.COEFF, inputs.DT_DZ)
    assert rel_err(host(u.grad), ubr) <= 1e-12
    assert rel_err(host(data.grad), dbr) <= 1e-12
    # the two stages separately compose to the same gradient
    u2 = torch.tensor(f.u, device=DEV, requires_grad=True)
    d2 = torch.tensor(f.data, device=DEV, requires_grad=True)
    x2 = autograd.vadv(autograd.hdiff(u2, inputs.COEFF), d2, w, inputs.DT_DZ)
    (x2 * ob).sum().backward()
    assert rel_err(host(x2), host(x)) <= 1e-14
    assert rel_err(host(u2.grad), host(u.grad)) <= 1e-13
    assert rel_err(host(d2.grad), host(data.grad)) <= 1e-13


# The gather's strips hold 60 output columns in FP64 and 124 in FP32 (two
# columns per lane), from i = -2, and 16 output rows from j = -2, of the
# padded domain: domains whose padded width or height ends exactly on, or one
# past, a strip edge of either width, plus the smallest ones.
STRIP_EDGE_CASES = [(56, 12, 2), (57, 13, 3), (116, 28, 2), (117, 29, 2), (55, 11, 2), (1, 2, 3), (2, 1, 2),
                    (176, 44, 1), (120, 12, 2), (121, 13, 2), (244, 5, 2), (245, 6, 2)]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("field", [False, True], ids=["scalar", "kappa"])
@pytest.mark.parametrize("dims", STRIP_EDGE_CASES, ids=lambda d: "x".join(map(str, d)))
def test_hdiff_adjoint_strip_edges(dims, field, dtype):
    ni, nj, nk = dims
    print(f"hdiff adjoint strip edges {dims} field={field} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=204)
    r = _ref(f, dtype)
    u = fields.from_padded(f.u, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask)
    lam = inputs.cotangent(ni, nj, nk)
    kap = inputs.coeff_field(ni, nj, nk) if field else None
    rr = (lambda a: round_f32(a)) if dtype == torch.float32 else (lambda a: a)
    lb = fields.from_interior(lam, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=9.0)
    before = ub.tensor.clone()
    o = api.Options(coeff_field=fields.from_interior(kap, dtype, DEV)) if field else None
    api.stencil_hdiff_adjoint(lb, mask, ub, dims, inputs.COEFF, opts=o)
    torch.cuda.synchronize()
    mx, my = orc.hdiff_masks(r.u, decide_f32=(dtype == torch.float32))
    ubr = orc.hdiff_adjoint(rr(lam), mx, my, c_scalar(inputs.COEFF, dtype), kappa=None if kap is None else rr(kap))
    assert rel_err(host(fields.padded(ub, ni, nj, nk)), ubr) <= TOL[dtype]
    # nothing outside the padded domain is written (row pitch, alignment offset)
    oi, oj, ok = ub.origin
    outside = torch.ones_like(before, dtype=torch.bool)
    outside[ok:ok + nk, oj - 2:oj + nj + 2, oi - 2:oi + ni + 2] = False
    assert torch.equal(ub.tensor[outside], before[outside])


LAMBDA_LAYOUT_CASES = [(67, 45, 7), (64, 20, 3), (125, 9, 2), (1, 5, 2), (248, 13, 2)]


@pytest.mark.parametrize("dims", LAMBDA_LAYOUT_CASES, ids=lambda d: "x".join(map(str, d)))
def test_hdiff_adjoint_f32_lambda_layouts(dims):
    """The binary32 gather reads a lane's two columns of lambda with one load
    where ni is even and lambda's rows keep 8-byte alignment, column by
    column otherwise (odd ni, odd pitch, a base 4 bytes off): every layout
    gives the same bits, and the oracle's values."""
    ni, nj, nk = dims
    print(f"hdiff adjoint FP32 lambda layouts {dims}", flush=True)
    dt = torch.float32
    f = inputs.fields_sized(ni, nj, nk, seed=205)
    u = fields.from_padded(f.u, dt, DEV)
    out = fields.alloc(ni, nj, nk, dt, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask)
    lam = inputs.cotangent(ni, nj, nk)
    # 8-byte aligned rows; an odd pitch (ni + 1 for even ni); a base 4 bytes off
    pitch = ni if ni % 2 else ni + 1
    t_odd = torch.zeros((nk, nj, pitch), dtype=dt, device=DEV)
    t_odd[:, :, :ni] = torch.as_tensor(lam).to(dt)
    t_off = torch.zeros((nk, nj, ni + 2), dtype=dt, device=DEV)
    t_off[:, :, 1:ni + 1] = torch.as_tensor(lam).to(dt)
    layouts = {"aligned": fields.from_interior(lam, dt, DEV),
               "odd_pitch": api.Field(t_odd, (0, 0, 0)),
               "offset": api.Field(t_off, (1, 0, 0))}
    res = {}
    for name, lb in layouts.items():
        ub = fields.alloc(ni, nj, nk, dt, DEV, fill=9.0)
        api.stencil_hdiff_adjoint(lb, mask, ub, dims, inputs.COEFF)
        torch.cuda.synchronize()
        res[name] = fields.padded(ub, ni, nj, nk).clone()
    assert torch.equal(res["aligned"], res["odd_pitch"]) and torch.equal(res["aligned"], res["offset"])
    mx, my = orc.hdiff_masks(round_f32(f.u), decide_f32=True)
    ubr = orc.hdiff_adjoint(round_f32(lam), mx, my, c_scalar(inputs.COEFF, dt))
    assert rel_err(host(res["aligned"]), ubr) <= TOL[dt]
