"""GPU parity of the generalised horizontal diffusion (a per-point
coefficient field and the damping form of the Laplacian) against the oracle:
hdiff and the fused step (values and limiter masks), their adjoints, the
coefficient-field gradient and the damping form's scalar coefficient
gradient, and a captured time loop against eager steps."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32, unpack_mask

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = [torch.float64, torch.float32]
IDS = ["f64", "f32"]
FORMS = [(api.HDIFF_DAMPING, False), (api.HDIFF_STATED, True), (api.HDIFF_DAMPING, True)]
FORM_IDS = ["damping", "kappa", "damping+kappa"]


def _r(a, dtype):
    return round_f32(a) if dtype == torch.float32 else a


def _opts(form, kappa_dev, **kw):
    return api.Options(hdiff_form=form, coeff_field=kappa_dev, **kw)


def _kappa(dims, dtype, with_field, child=103):
    ni, nj, nk = dims
    if not with_field:
        return None, None
    k = inputs.coeff_field(ni, nj, nk, child=child)
    return k, fields.from_interior(k, dtype, DEV)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("form,field", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("tile", [64, 32, 16])
@pytest.mark.parametrize("dims", [(67, 45, 7), (1, 1, 3), (130, 5, 4)], ids=lambda d: "x".join(map(str, d)))
def test_hdiff_general(dims, tile, form, field, dtype):
    ni, nj, nk = dims
    print(f"general hdiff {dims} tile={tile} form={form} field={field} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=600)
    k, kd = _kappa(dims, dtype, field)
    u = fields.from_padded(f.u, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    o = _opts(form, kd, tile_i=tile)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask, opts=o)
    torch.cuda.synchronize()
    want, mx, my = orc.hdiff(_r(f.u, dtype), c_scalar(inputs.COEFF, dtype), decide_f32=(dtype == torch.float32),
                             kappa=None if k is None else _r(k, dtype), damping=(form == api.HDIFF_DAMPING))
    assert rel_err(host(fields.interior(out, ni, nj, nk)), want[:, 2:-2, 2:-2]) <= TOL[dtype]
    gx, gy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gx, mx) and np.array_equal(gy, my)


STEP_CASES = [(64, 64, 16), (67, 45, 7), (1, 1, 1), (33, 17, 137), (3, 70, 97), (130, 3, 144)]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("form,field", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("dims", STEP_CASES, ids=lambda d: "x".join(map(str, d)))
def test_step_general(dims, form, field, dtype):
    ni, nj, nk = dims
    print(f"general step {dims} form={form} field={field} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=601)
    k, kd = _kappa(dims, dtype, field)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-3.0)
    mask = fields.mask_tensor(dims, DEV)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=_opts(form, kd))
    torch.cuda.synchronize()
    nxt, mx, my = orc.step(_r(f.u, dtype), _r(f.data, dtype), _r(f.w, dtype), c_scalar(inputs.COEFF, dtype),
                           inputs.DT_DZ, decide_f32=(dtype == torch.float32),
                           kappa=None if k is None else _r(k, dtype), damping=(form == api.HDIFF_DAMPING))
    got = host(fields.padded(out, ni, nj, nk))
    assert rel_err(got[:, 2:-2, 2:-2], nxt[:, 2:-2, 2:-2]) <= TOL[dtype]
    # the halo of out is not written
    ring = np.ones(got.shape, bool)
    ring[:, 2:-2, 2:-2] = False
    assert np.all(got[ring] == -3.0)
    gx, gy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gx, mx) and np.array_equal(gy, my)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("tile", [64, 32, 16])
def test_step_general_128_column_tiles(tile, dtype):
    """The generalised step (damping form, coefficient field) in 128-column
    tiles equals the 256-column tiles bit for bit, masks included, and the
    oracle."""
    dims = (67, 45, 33)
    ni, nj, nk = dims
    print(f"general step 128-column tiles {tile}x{128 // tile} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=603)
    k, kd = _kappa(dims, dtype, True)
    u, data, w = dev_fields(f, dtype, DEV)
    res = {}
    for tj in (128 // tile, 256 // tile):
        out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-3.0)
        mask = fields.mask_tensor(dims, DEV)
        o = _opts(api.HDIFF_DAMPING, kd, tile_i=tile, tile_j=tj)
        api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=o)
        torch.cuda.synchronize()
        res[tj] = (fields.padded(out, ni, nj, nk).clone(), mask.clone())
    a, b = res[128 // tile], res[256 // tile]
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    nxt, mx, my = orc.step(_r(f.u, dtype), _r(f.data, dtype), _r(f.w, dtype), c_scalar(inputs.COEFF, dtype),
                           inputs.DT_DZ, decide_f32=(dtype == torch.float32), kappa=_r(k, dtype), damping=True)
    assert rel_err(host(a[0][:, 2:-2, 2:-2]), nxt[:, 2:-2, 2:-2]) <= TOL[dtype]
    gx, gy = unpack_mask(a[1], ni, nj, nk)
    assert np.array_equal(gx, mx) and np.array_equal(gy, my)


def test_step_general_full_size():
    """512 x 512 x 80 FP64, damping form with a coefficient field."""
    dims = (512, 512, 80)
    ni, nj, nk = dims
    f = inputs.fields_for(inputs.STEP_512)
    k, kd = _kappa(dims, torch.float64, True)
    u, data, w = dev_fields(f, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, opts=_opts(api.HDIFF_DAMPING, kd))
    torch.cuda.synchronize()
    nxt, _, _ = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ, kappa=k, damping=True)
    assert rel_err(host(fields.interior(out, ni, nj, nk)), nxt[:, 2:-2, 2:-2]) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("form,field", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("dims", [(67, 45, 7), (1, 1, 1), (33, 17, 137), (130, 3, 20)],
                         ids=lambda d: "x".join(map(str, d)))
def test_step_adjoint_general(dims, form, field, dtype):
    """The GPU's own masks feed the oracle, so the linear maps are compared."""
    ni, nj, nk = dims
    print(f"general step adjoint {dims} form={form} field={field} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=602)
    k, kd = _kappa(dims, dtype, field)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    o = _opts(form, kd)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=o)
    ob = inputs.cotangent(ni, nj, nk)
    xb = fields.from_interior(ob, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=123.0)
    db = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    api.stencil_step_adjoint(xb, w, mask, ub, db, dims, inputs.COEFF, inputs.DT_DZ, opts=o)
    torch.cuda.synchronize()
    mx, my = unpack_mask(mask, ni, nj, nk)
    ubr, dbr = orc.step_adjoint(_r(ob, dtype), _r(f.w, dtype), mx, my, c_scalar(inputs.COEFF, dtype),
                                inputs.DT_DZ, kappa=None if k is None else _r(k, dtype),
                                damping=(form == api.HDIFF_DAMPING))
    assert rel_err(host(fields.padded(ub, ni, nj, nk)), ubr) <= TOL[dtype]
    assert rel_err(host(fields.interior(db, ni, nj, nk)), dbr) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("tile", [64, 32, 16])
def test_hdiff_adjoint_general(tile, dtype):
    ni, nj, nk = 75, 41, 6
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=603)
    k, kd = _kappa(dims, dtype, True)
    u = fields.from_padded(f.u, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor(dims, DEV)
    o = _opts(api.HDIFF_DAMPING, kd, tile_i=tile)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask, opts=o)
    lam = inputs.cotangent(ni, nj, nk)
    lb = fields.from_interior(lam, dtype, DEV)
    ub = fields.alloc(ni, nj, nk, dtype, DEV, fill=7.0)
    api.stencil_hdiff_adjoint(lb, mask, ub, dims, inputs.COEFF, opts=o)
    torch.cuda.synchronize()
    mx, my = unpack_mask(mask, ni, nj, nk)
    want = orc.hdiff_adjoint(_r(lam, dtype), mx, my, c_scalar(inputs.COEFF, dtype), kappa=_r(k, dtype),
                             damping=True)
    assert rel_err(host(fields.padded(ub, ni, nj, nk)), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("form", [api.HDIFF_STATED, api.HDIFF_DAMPING], ids=["stated", "damping"])
@pytest.mark.parametrize("dims", [(64, 64, 16), (67, 45, 7), (1, 1, 1), (130, 3, 20)],
                         ids=lambda d: "x".join(map(str, d)))
def test_coefficient_gradients(dims, form, dtype):
    """kappa_bar = -lam D(u) point by point, and the damping form's scalar
    coeff_bar, both fed the same u and lam as the oracle."""
    ni, nj, nk = dims
    f = inputs.fields_sized(ni, nj, nk, seed=604)
    lam = inputs.cotangent(ni, nj, nk)
    u = fields.from_padded(f.u, dtype, DEV)
    lb = fields.from_interior(lam, dtype, DEV)
    kb = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=5.0)
    o = api.Options(hdiff_form=form)
    api.stencil_coeff_field_adjoint(u, lb, kb, dims, opts=o)
    cb = torch.full((1,), 9.0, dtype=torch.float64, device=DEV)
    n = api.stencil_param_workspace_bytes(dtype, dims)
    ws = torch.empty(n, dtype=torch.uint8, device=DEV) if n else None
    api.stencil_step_param_adjoint(u, None, None, lb, None, cb, dims, inputs.DT_DZ, ws=ws, opts=o)
    torch.cuda.synchronize()
    damping = form == api.HDIFF_DAMPING
    ur, lr = _r(f.u, dtype), _r(lam, dtype)
    mx, my = orc.hdiff_masks(ur, decide_f32=(dtype == torch.float32), damping=damping)
    want = orc.coeff_field_grad(ur, lr, mx, my, damping=damping)
    assert rel_err(host(fields.interior(kb, ni, nj, nk)), want) <= TOL[dtype]
    g = orc.coeff_grad(ur, lr, mx, my, damping=damping)
    scale = float(np.sum(np.abs(want))) or 1.0
    assert abs(float(cb.item()) - g) <= TOL[dtype] * scale, (cb.item(), g)


def test_general_graph_matches_eager():
    """A captured 6-step loop of the damping form with a coefficient field
    equals 6 eager steps bit for bit (the graph reads the field at replay)."""
    dtype = torch.float64
    ni, nj, nk = 96, 80, 24
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=605)
    k, kd = _kappa(dims, dtype, True)
    o = _opts(api.HDIFF_DAMPING, kd)
    data = fields.from_interior(f.data, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    e = [fields.from_padded(f.u, dtype, DEV), fields.from_padded(f.u, dtype, DEV)]
    for n in range(6):
        api.stencil_step(e[n % 2], data, w, e[(n + 1) % 2], dims, inputs.COEFF, inputs.DT_DZ, opts=o)
    torch.cuda.synchronize()
    eager = host(fields.padded(e[0], ni, nj, nk))
    u_a = fields.from_padded(f.u, dtype, DEV)
    u_b = fields.from_padded(f.u, dtype, DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = api.stencil_graph_capture_steps(6, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ, opts=o,
                                            stream=s)
    try:
        for _ in range(2):  # replays start from the state the last one left: reset in between
            u_a.tensor.copy_(fields.from_padded(f.u, dtype, DEV).tensor)
            torch.cuda.synchronize()
            api.stencil_graph_launch(g, stream=s)
            s.synchronize()
            assert np.array_equal(host(fields.padded(u_a, ni, nj, nk)), eager)
    finally:
        api.stencil_graph_destroy(g)


def test_autograd_step_with_field_and_damping():
    """autograd.step with a per-point coefficient tensor and the damping
    form: the gradients are the adjoint entry points' (bit for bit) and match
    the oracle's (kappa_bar = -lam D(u), lam = T^-T x_bar)."""
    from paper_2311_08322_amd import autograd
    ni, nj, nk = 40, 24, 12
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=606)
    k = inputs.coeff_field(ni, nj, nk)
    dt = torch.float64
    u = torch.tensor(f.u, dtype=dt, device=DEV, requires_grad=True)
    data = torch.tensor(f.data, dtype=dt, device=DEV, requires_grad=True)
    w = torch.tensor(f.w, dtype=dt, device=DEV, requires_grad=True)
    kap = torch.tensor(k, dtype=dt, device=DEV, requires_grad=True)
    ob = inputs.cotangent(ni, nj, nk)
    x = autograd.step(u, data, w, kap, inputs.DT_DZ, damping=True)
    (x * torch.tensor(ob, dtype=dt, device=DEV)).sum().backward()
    nxt, mx, my = orc.step(f.u, f.data, f.w, 0.0, inputs.DT_DZ, kappa=k, damping=True)
    assert rel_err(host(x), nxt[:, 2:-2, 2:-2]) <= 1e-12
    lam = orc.vadv_adjoint(ob, f.w, inputs.DT_DZ)
    assert rel_err(host(data.grad), lam) <= 1e-12
    ubr = orc.hdiff_adjoint(lam, mx, my, 0.0, kappa=k, damping=True)
    assert rel_err(host(u.grad), ubr) <= 1e-12
    assert rel_err(host(kap.grad), orc.coeff_field_grad(f.u, lam, mx, my, damping=True)) <= 1e-12
    assert rel_err(host(w.grad), orc.w_grad(f.w, nxt[:, 2:-2, 2:-2], lam, inputs.DT_DZ)) <= 1e-12


@pytest.mark.parametrize("field", [False, True], ids=["scalar", "field"])
def test_autograd_hdiff_coefficient_gradient(field):
    from paper_2311_08322_amd import autograd
    ni, nj, nk = 37, 29, 5
    f = inputs.fields_sized(ni, nj, nk, seed=607)
    k = inputs.coeff_field(ni, nj, nk)
    dt = torch.float64
    u = torch.tensor(f.u, dtype=dt, device=DEV, requires_grad=True)
    c = torch.tensor(k if field else inputs.COEFF, dtype=dt, device=DEV, requires_grad=True)
    ob = inputs.cotangent(ni, nj, nk)
    out = autograd.hdiff(u, c, damping=True)
    (out * torch.tensor(ob, dtype=dt, device=DEV)).sum().backward()
    mx, my = orc.hdiff_masks(f.u, damping=True)
    want_u = orc.hdiff_adjoint(ob, mx, my, inputs.COEFF, kappa=k if field else None, damping=True)
    assert rel_err(host(u.grad), want_u) <= 1e-12
    if field:
        assert rel_err(host(c.grad), orc.coeff_field_grad(f.u, ob, mx, my, damping=True)) <= 1e-12
    else:
        g = orc.coeff_grad(f.u, ob, mx, my, damping=True)
        scale = float(np.sum(np.abs(orc.coeff_field_grad(f.u, ob, mx, my, damping=True))))
        assert abs(float(c.grad.item()) - g) <= 1e-12 * scale


def test_autotune_hdiff_damping():
    """The tuner times hdiff's tile candidates in the damping form (the only
    hdiff with a tile); the tuned tile then serves that form's calls."""
    dims = (67, 45, 7)
    ni, nj, nk = dims
    best = api.stencil_autotune(torch.float64, api.OP_HDIFF, dims, reps=2)
    assert best > 0
    ti, tj, _, _ = api.stencil_tuning_lookup(torch.float64, api.OP_HDIFF, dims)
    assert (ti, tj) in ((64, 4), (32, 8), (16, 16))
    f = inputs.fields_sized(ni, nj, nk, seed=601)
    u = fields.from_padded(f.u, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, opts=api.Options(hdiff_form=api.HDIFF_DAMPING))
    torch.cuda.synchronize()
    want, _, _ = orc.hdiff(f.u, inputs.COEFF, damping=True)
    assert rel_err(host(fields.interior(out, ni, nj, nk)), want[:, 2:-2, 2:-2]) <= TOL[torch.float64]
