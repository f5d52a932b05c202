"""GPU parity of the forward stencils against the CPU oracle.

Element-by-element on the same seeded inputs; masks bit-exact; values
within 1e-12 (FP64) or 2e-5 (FP32, against the FP64 oracle run on the
binary32-rounded inputs with its limiter decisions taken in binary32)
relative in the infinity norm.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32, unpack_mask

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = [torch.float64, torch.float32]


def _ref_inputs(f, dtype):
    if dtype == torch.float32:
        return inputs.Fields(u=round_f32(f.u), w=round_f32(f.w), data=round_f32(f.data))
    return f


def _opts(impl, tile=0, col=0, dtype=torch.float64, dom=None, op=api.OP_STEP, order=api.ORDER_AUTO):
    o = api.Options(impl=impl, tile_i=tile, tile_j=(256 // tile if tile else 0), column_store=col, tile_order=order)
    if impl == api.IMPL_PLAIN or (dom is not None and dom[2] > api.stencil_max_fused_nk()):
        o.workspace = fields.workspace(op, dtype, dom, o)
    return o


# ------------------------------------------------------------------ hdiff
# the standalone hdiff walks strips of 56 (FP64) or 120 (FP32) columns and
# 16 rows: domains ending on and one past those edges too
HDIFF_CASES = [(64, 64, 16), (67, 45, 7), (1, 1, 1), (130, 3, 5), (5, 130, 3), (2, 2, 2), (56, 16, 2), (57, 17, 2),
               (120, 9, 2), (121, 33, 2), (240, 3, 2), (241, 5, 2)]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("impl,tile", [(api.IMPL_PLAIN, 0), (api.IMPL_FUSED, 64), (api.IMPL_FUSED, 32),
                                       (api.IMPL_FUSED, 16)], ids=["plain", "t64", "t32", "t16"])
@pytest.mark.parametrize("dims", HDIFF_CASES, ids=lambda d: "x".join(map(str, d)))
def test_hdiff(dims, impl, tile, dtype):
    ni, nj, nk = dims
    print(f"hdiff {dims} impl={impl} tile={tile} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=101)
    r = _ref_inputs(f, dtype)
    u = fields.from_padded(f.u, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-7.0)
    mask = fields.mask_tensor(dims, DEV)
    coeff = c_scalar(inputs.COEFF, dtype)
    api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask, opts=_opts(impl, tile, 0, dtype, dims, api.OP_HDIFF))
    torch.cuda.synchronize()
    ref, mx, my = orc.hdiff(r.u, coeff, decide_f32=(dtype == torch.float32))
    got = host(fields.interior(out, ni, nj, nk))
    assert rel_err(got, ref[:, 2:-2, 2:-2]) <= TOL[dtype]
    gmx, gmy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gmx, mx) and np.array_equal(gmy, my)
    # the halo of out is untouched
    full = host(fields.padded(out, ni, nj, nk))
    ring = np.ones(full.shape, bool)
    ring[:, 2:-2, 2:-2] = False
    assert np.all(full[ring] == -7.0)


def test_hdiff_config1_without_mask():
    ni, nj, nk = inputs.HDIFF_64.ni, inputs.HDIFF_64.nj, inputs.HDIFF_64.nk
    f = inputs.fields_for(inputs.HDIFF_64)
    u = fields.from_padded(f.u, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, fill=0.0)
    api.stencil_hdiff(u, out, (ni, nj, nk), inputs.COEFF)
    ref, _, _ = orc.hdiff(f.u, inputs.COEFF)
    assert rel_err(host(fields.interior(out, ni, nj, nk)), ref[:, 2:-2, 2:-2]) <= 1e-12


# ------------------------------------------------------------------ vadv
VADV_NK = [1, 2, 16, 17, 80, 96, 97, 128, 137, 160, 161, 200]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("impl", [api.IMPL_AUTO, api.IMPL_PLAIN], ids=["auto", "plain"])
@pytest.mark.parametrize("nk", VADV_NK)
def test_vadv(nk, impl, dtype):
    ni, nj = 70, 9
    print(f"vadv nk={nk} impl={impl} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=102)
    r = _ref_inputs(f, dtype)
    uin = fields.from_interior(f.u[:, 2:-2, 2:-2], dtype, DEV)
    data = fields.from_interior(f.data, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    dom = (ni, nj, nk)
    api.stencil_vadv(uin, data, w, out, dom, inputs.DT_DZ, opts=_opts(impl, 0, 0, dtype, dom, api.OP_VADV))
    torch.cuda.synchronize()
    ref = orc.vadv(r.u[:, 2:-2, 2:-2], r.data, r.w, inputs.DT_DZ)
    assert rel_err(host(fields.interior(out, ni, nj, nk)), ref) <= TOL[dtype]


def test_vadv_full_size_residual():
    """256x256x80 FP64: oracle parity and the GPU solution's own residual."""
    wl = inputs.STEP_256
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    f = inputs.fields_for(wl)
    uin = fields.from_interior(f.u[:, 2:-2, 2:-2], torch.float64, DEV)
    data = fields.from_interior(f.data, torch.float64, DEV)
    w = fields.from_interior(f.w, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    api.stencil_vadv(uin, data, w, out, (ni, nj, nk), inputs.DT_DZ)
    x = host(fields.interior(out, ni, nj, nk))
    ref = orc.vadv(f.u[:, 2:-2, 2:-2], f.data, f.w, inputs.DT_DZ)
    assert rel_err(x, ref) <= 1e-12
    res = orc.tridiag_apply(x, f.w, inputs.DT_DZ) - (f.u[:, 2:-2, 2:-2] + f.data)
    assert np.max(np.abs(res)) < 1e-13


# ------------------------------------------------------------------ step
# column lengths at the FP64 register classes' edges too: 88 and 96 (half
# columns of 48 levels), 97 and 144 (the 128-column long form)
STEP_CASES = [(64, 64, 16), (100, 37, 80), (67, 45, 7), (1, 1, 1), (9, 5, 2), (30, 70, 79), (33, 17, 137),
              (20, 20, 161), (45, 21, 88), (37, 19, 96), (29, 23, 97), (21, 13, 144)]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("impl,tile,col,order", [
    (api.IMPL_PLAIN, 0, 0, 0),
    (api.IMPL_FUSED, 64, api.COLUMN_REGISTERS, 0), (api.IMPL_FUSED, 64, api.COLUMN_OUTBUF, 0),
    (api.IMPL_FUSED, 32, api.COLUMN_REGISTERS, 0), (api.IMPL_FUSED, 16, api.COLUMN_OUTBUF, 0),
    (api.IMPL_FUSED, 64, api.COLUMN_SPLIT, api.ORDER_XCD), (api.IMPL_FUSED, 32, api.COLUMN_SPLIT, api.ORDER_XCD),
    (api.IMPL_FUSED, 16, api.COLUMN_SPLIT, api.ORDER_XCD), (api.IMPL_FUSED, 64, api.COLUMN_SPLIT, api.ORDER_DISPATCH),
    (api.IMPL_FUSED, 32, api.COLUMN_SPLIT, api.ORDER_DISPATCH), (api.IMPL_AUTO, 0, 0, 0)],
    ids=["plain", "t64reg", "t64out", "t32reg", "t16out", "t64split", "t32split", "t16split", "t64split_dispatch",
         "t32split_dispatch", "auto"])
@pytest.mark.parametrize("dims", STEP_CASES, ids=lambda d: "x".join(map(str, d)))
def test_step(dims, impl, tile, col, order, dtype):
    ni, nj, nk = dims
    if nk > api.stencil_max_fused_nk() and impl == api.IMPL_FUSED:
        pytest.skip("longer than the fused classes (covered by plain/auto)")
    print(f"step {dims} impl={impl} tile={tile} col={col} order={order} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=103)
    r = _ref_inputs(f, dtype)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-3.0)
    mask = fields.mask_tensor(dims, DEV)
    coeff = c_scalar(inputs.COEFF, dtype)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask,
                     opts=_opts(impl, tile, col, dtype, dims, api.OP_STEP, order))
    torch.cuda.synchronize()
    ref, mx, my = orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=(dtype == torch.float32))
    assert rel_err(host(fields.interior(out, ni, nj, nk)), ref[:, 2:-2, 2:-2]) <= TOL[dtype]
    gmx, gmy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gmx, mx) and np.array_equal(gmy, my)
    full = host(fields.padded(out, ni, nj, nk))
    ring = np.ones(full.shape, bool)
    ring[:, 2:-2, 2:-2] = False
    assert np.all(full[ring] == -3.0)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("tile", [64, 32, 16])
@pytest.mark.parametrize("dims", [(100, 37, 80), (67, 45, 7), (1, 1, 1), (30, 70, 79), (33, 17, 137),
                                  (21, 13, 144), (45, 21, 88)], ids=lambda d: "x".join(map(str, d)))
def test_step_128_column_tiles(dims, tile, dtype):
    """The two-ended step in 128-column tiles (256-lane workgroups): the
    oracle's values, its masks bit for bit, and the same bits as the
    256-column tile of the same width."""
    ni, nj, nk = dims
    if nk > api.stencil_max_fused_nk(api.F64 if dtype == torch.float64 else api.F32):
        pytest.skip("longer than the fused classes")
    print(f"step 128-column tiles {dims} tile {tile}x{128 // tile} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=107)
    r = _ref_inputs(f, dtype)
    u, data, w = dev_fields(f, dtype, DEV)
    res = {}
    for tj in (128 // tile, 256 // tile):
        out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-3.0)
        mask = fields.mask_tensor(dims, DEV)
        o = api.Options(impl=api.IMPL_FUSED, tile_i=tile, tile_j=tj, column_store=api.COLUMN_SPLIT)
        api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask, opts=o)
        torch.cuda.synchronize()
        res[tj] = (fields.padded(out, ni, nj, nk).clone(), mask.clone())
    a, b = res[128 // tile], res[256 // tile]
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    ref, mx, my = orc.step(r.u, r.data, r.w, c_scalar(inputs.COEFF, dtype), inputs.DT_DZ,
                           decide_f32=(dtype == torch.float32))
    assert rel_err(host(a[0][:, 2:-2, 2:-2]), ref[:, 2:-2, 2:-2]) <= TOL[dtype]
    gmx, gmy = unpack_mask(a[1], ni, nj, nk)
    assert np.array_equal(gmx, mx) and np.array_equal(gmy, my)


def test_step_unaligned_and_strided_layouts():
    """Fields with different pitches, origins and an offset vertical interval."""
    ni, nj, nk = 77, 23, 19
    f = inputs.fields_sized(ni, nj, nk, seed=104)
    # u embedded in a bigger allocation: 3 extra levels below, odd pitch
    big = torch.zeros((nk + 5, nj + 9, ni + 13), dtype=torch.float64, device=DEV)
    big[3:3 + nk, 4 - 2:4 + nj + 2, 5 - 2:5 + ni + 2] = torch.as_tensor(f.u, device=DEV)
    u = api.Field(big, (5, 4, 3))
    data = fields.from_interior(f.data, torch.float64, DEV, aligned=False)
    w = fields.from_interior(f.w, torch.float64, DEV, aligned=False)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, aligned=False, fill=0.0)
    api.stencil_step(u, data, w, out, (ni, nj, nk), inputs.COEFF, inputs.DT_DZ)
    ref, _, _ = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    assert rel_err(host(fields.interior(out, ni, nj, nk)), ref[:, 2:-2, 2:-2]) <= 1e-12


@pytest.mark.parametrize("dims", [(64, 20, 3), (248, 13, 2), (67, 9, 2), (2, 5, 2)],
                         ids=lambda d: "x".join(map(str, d)))
def test_hdiff_f32_layouts(dims):
    """The binary32 row walk reads and writes column pairs with one 8-byte
    access where ni is even and the rows of u and out keep 8-byte alignment,
    column by column otherwise (odd ni, u 4 bytes off, out with an odd
    pitch): the same bits, the same masks, and the oracle's values."""
    ni, nj, nk = dims
    print(f"hdiff FP32 layouts {dims}", flush=True)
    dt = torch.float32
    f = inputs.fields_sized(ni, nj, nk, seed=106)
    ua = fields.from_padded(f.u, dt, DEV)
    big = torch.zeros((nk, nj + 4, ni + 5), dtype=dt, device=DEV)
    big[:, :, 1:ni + 5] = torch.as_tensor(f.u).to(dt)
    uo = api.Field(big, (3, 2, 0))  # the padded corner 4 bytes past an 8-byte boundary
    runs = {}
    for name, u, aligned_out in (("aligned", ua, True), ("u_off", uo, True), ("out_odd", ua, False)):
        if aligned_out:
            out = fields.alloc(ni, nj, nk, dt, DEV, fill=0.0)
        else:
            pitch = ni + 5 if (ni + 4) % 2 == 0 else ni + 4
            out = api.Field(torch.zeros((nk, nj + 4, pitch), dtype=dt, device=DEV), (2, 2, 0))
        mask = fields.mask_tensor(dims, DEV)
        api.stencil_hdiff(u, out, dims, inputs.COEFF, mask=mask)
        torch.cuda.synchronize()
        runs[name] = (fields.interior(out, ni, nj, nk).clone(), mask.clone())
    for name in ("u_off", "out_odd"):
        assert torch.equal(runs[name][0], runs["aligned"][0]), name
        assert torch.equal(runs[name][1], runs["aligned"][1]), name
    ref, mx, my = orc.hdiff(round_f32(f.u), c_scalar(inputs.COEFF, dt), decide_f32=True)
    assert rel_err(host(runs["aligned"][0]), ref[:, 2:-2, 2:-2]) <= TOL[dt]
    gx, gy = unpack_mask(runs["aligned"][1], ni, nj, nk)
    assert np.array_equal(gx, mx) and np.array_equal(gy, my)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("wl", [inputs.STEP_256, inputs.STEP_512], ids=["256", "512"])
def test_step_full_size(wl, dtype):
    """The benchmark workloads at full size in the launch configuration the
    benchmark times (fused, default tile), every output element checked."""
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    print(f"step full {wl.name} {dtype}", flush=True)
    f = inputs.fields_for(wl)
    r = _ref_inputs(f, dtype)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
    mask = fields.mask_tensor((ni, nj, nk), DEV)
    api.stencil_step(u, data, w, out, (ni, nj, nk), inputs.COEFF, inputs.DT_DZ, mask=mask)
    torch.cuda.synchronize()
    ref, mx, my = orc.step(r.u, r.data, r.w, c_scalar(inputs.COEFF, dtype), inputs.DT_DZ,
                           decide_f32=(dtype == torch.float32))
    assert rel_err(host(fields.interior(out, ni, nj, nk)), ref[:, 2:-2, 2:-2]) <= TOL[dtype]
    gmx, gmy = unpack_mask(mask, ni, nj, nk)
    assert np.array_equal(gmx, mx) and np.array_equal(gmy, my)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("tile", [64, 32, 16])
def test_step_tile_orders_agree_full_size(tile, dtype):
    """Both tile orders compute every column with the same operations: the
    512x512x80 step and its masks agree bit for bit between them."""
    wl = inputs.STEP_512
    dims = (wl.ni, wl.nj, wl.nk)
    print(f"step tile orders {dims} tile {tile} {dtype}", flush=True)
    f = inputs.fields_for(wl)
    u, data, w = dev_fields(f, dtype, DEV)
    res = []
    for order in (api.ORDER_XCD, api.ORDER_DISPATCH):
        out = fields.alloc(*dims, dtype, DEV, fill=0.0)
        mask = fields.mask_tensor(dims, DEV)
        api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, mask=mask,
                         opts=_opts(api.IMPL_FUSED, tile, api.COLUMN_SPLIT, dtype, dims, api.OP_STEP, order))
        res.append((out, mask))
    torch.cuda.synchronize()
    assert torch.equal(fields.interior(res[0][0], *dims), fields.interior(res[1][0], *dims))
    assert torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_autotune_step_and_tuned_step(dtype):
    """The step's autotuner records a supported tile, column store and tile
    order for the size class, and the step run with the tuned entry matches
    the oracle."""
    dims = (150, 70, 40)
    print(f"autotune step {dims} {dtype}", flush=True)
    api.stencil_clear_tuning()
    best = api.stencil_autotune(dtype, api.OP_STEP, dims, reps=2)
    assert best > 0
    ti, tj, col, order = api.stencil_tuning_lookup(dtype, api.OP_STEP, dims)
    assert (ti, tj) in ((64, 4), (32, 8), (16, 16)) or ((ti, tj) in ((64, 2), (32, 4), (16, 8)) and
                                                        col == api.COLUMN_SPLIT)
    assert col in (api.COLUMN_REGISTERS, api.COLUMN_OUTBUF, api.COLUMN_SPLIT)
    assert order in (api.ORDER_XCD, api.ORDER_DISPATCH)
    f = inputs.fields_sized(*dims, seed=108)
    r = _ref_inputs(f, dtype)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(*dims, dtype, DEV, fill=0.0)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ)
    torch.cuda.synchronize()
    ref, _, _ = orc.step(r.u, r.data, r.w, c_scalar(inputs.COEFF, dtype), inputs.DT_DZ,
                         decide_f32=(dtype == torch.float32))
    assert rel_err(host(fields.interior(out, *dims)), ref[:, 2:-2, 2:-2]) <= TOL[dtype]
    api.stencil_clear_tuning()


def test_autotune_on_fields_then_step():
    """Tuning on the caller's fields leaves the inputs as they were, records
    a supported entry, and the step with it matches the oracle."""
    dims = (130, 90, 60)
    print(f"autotune on fields {dims}", flush=True)
    api.stencil_clear_tuning()
    f = inputs.fields_sized(*dims, seed=109)
    u, data, w = dev_fields(f, torch.float64, DEV)
    u0 = u.tensor.clone()
    scratch = fields.alloc(*dims, torch.float64, DEV, fill=0.0)
    assert api.stencil_autotune_fields(u, data, w, scratch, dims, reps=2) > 0
    assert torch.equal(u.tensor, u0)
    ti, tj, col, order = api.stencil_tuning_lookup(torch.float64, api.OP_STEP, dims)
    assert ((ti, tj) in ((64, 4), (32, 8), (16, 16)) or (ti, tj) in ((64, 2), (32, 4), (16, 8))) and \
        order in (api.ORDER_XCD, api.ORDER_DISPATCH)
    out = fields.alloc(*dims, torch.float64, DEV, fill=0.0)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ)
    torch.cuda.synchronize()
    ref, _, _ = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    assert rel_err(host(fields.interior(out, *dims)), ref[:, 2:-2, 2:-2]) <= 1e-12
    api.stencil_clear_tuning()


def test_empty_domains_leave_outputs_alone():
    f = inputs.fields_sized(8, 8, 4, seed=105)
    u, data, w = dev_fields(f, torch.float64, DEV)
    out = fields.alloc(8, 8, 4, torch.float64, DEV, fill=5.0)
    for dom in [(0, 8, 4), (8, 0, 4), (8, 8, 0)]:
        api.stencil_step(u, data, w, out, dom, inputs.COEFF, inputs.DT_DZ)
        api.stencil_hdiff(u, out, dom, inputs.COEFF)
    torch.cuda.synchronize()
    assert torch.all(out.tensor == 5.0)
