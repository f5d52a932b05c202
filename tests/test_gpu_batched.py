"""GPU parity of the persistent batched launches.

The uneven 32-field workload (inputs.batch_fields: ni, nj in [48, 384], nk
in [40, 137] inclusive) runs as one forward launch and one adjoint pair; every field
is checked against the oracle, and bit for bit against separate
single-field launches, which solve each column with the same two-ended
elimination.  Masks are compared bit for bit.  Smaller batches cover empty
and degenerate fields, items without masks, the column limit, repeated
calls and replay from a captured graph.
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
IDS = ["f64", "f32"]


def _ref(f, dtype):
    if dtype == torch.float32:
        return inputs.Fields(u=round_f32(f.u), w=round_f32(f.w), data=round_f32(f.data))
    return f


@pytest.fixture(scope="module")
def batch():
    return inputs.batch_fields()


_ORACLE = {}


def _oracle_forward(batch, dtype):
    """Per field: (next padded state, mx, my) from the oracle (cached)."""
    key = ("fwd", dtype)
    if key not in _ORACLE:
        coeff = c_scalar(inputs.COEFF, dtype)
        res = []
        for ni, nj, nk, f in batch:
            r = _ref(f, dtype)
            res.append(orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=(dtype == torch.float32)))
        _ORACLE[key] = res
    return _ORACLE[key]


def _storage(ni, nj, nk):
    """Storage extents of a field whose domain may be empty: at least one
    point along each axis (a field's data pointer may not be NULL)."""
    return max(ni, 1), max(nj, 1), max(nk, 1)


def _items(batch, dtype, masks=True):
    """Device fields of a batch (fields drawn at their storage extents)."""
    items = []
    for ni, nj, nk, f in batch:
        u, data, w = dev_fields(f, dtype, DEV)
        dims = (ni, nj, nk)
        out = fields.alloc(*_storage(ni, nj, nk), dtype, DEV, fill=0.0)
        items.append(dict(u=u, data=data, w=w, out=out, domain=dims,
                          coeff=inputs.COEFF, dt_dz=inputs.DT_DZ,
                          mask=fields.mask_tensor(dims, DEV) if masks else None))
    return items


def _ws(n):
    return torch.empty(max(n, 1), dtype=torch.uint8, device=DEV) if n else None


def _run_batched(items, dtype, tile=0):
    ws = _ws(api.stencil_batch_workspace_bytes(dtype, items))
    api.stencil_step_batched(dtype, items, ws, opts=api.Options(tile_i=tile))
    return ws


def _interior(it):
    ni, nj, nk = it["domain"]
    return fields.interior(it["out"], ni, nj, nk)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
def test_forward_batch_vs_oracle(batch, dtype):
    print(f"batched forward, 32 fields, {dtype}", flush=True)
    items = _items(batch, dtype)
    _run_batched(items, dtype)
    torch.cuda.synchronize()
    ref = _oracle_forward(batch, dtype)
    for it, (nxt, mx, my) in zip(items, ref):
        ni, nj, nk = it["domain"]
        err = rel_err(host(_interior(it)), nxt[:, 2:-2, 2:-2])
        assert err <= TOL[dtype], (it["domain"], err)
        gx, gy = unpack_mask(it["mask"], ni, nj, nk)
        assert np.array_equal(gx, mx) and np.array_equal(gy, my), it["domain"]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("tile", [64, 32, 16])
def test_forward_batch_vs_separate(batch, dtype, tile):
    print(f"batched forward vs separate launches, tile {tile}, {dtype}", flush=True)
    items = _items(batch, dtype)
    _run_batched(items, dtype, tile)
    sep = _items(batch, dtype)
    for it in sep:
        o = api.Options(tile_i=tile)
        o.workspace = fields.workspace(api.OP_STEP, dtype, it["domain"], o)
        api.stencil_step(it["u"], it["data"], it["w"], it["out"], it["domain"], inputs.COEFF, inputs.DT_DZ,
                         mask=it["mask"], opts=o)
    torch.cuda.synchronize()
    for a, b in zip(items, sep):
        assert torch.equal(_interior(a), _interior(b)), a["domain"]
        assert torch.equal(a["mask"], b["mask"]), a["domain"]


def _least_cost_tile(ni, nj, nt, dtype):
    """The tile width an automatic batch gives a field without a tuned entry:
    the lanes its tiles span (idle edge lanes included) times a per-width
    cost (relative to 64-wide tiles), least first, ties to the wider."""
    fac = {64: 1000, 32: 1000, 16: 1060} if dtype == torch.float64 else {64: 1000, 32: 1080, 16: 1250}
    best, least = 64, None
    for w in (64, 32, 16):
        h = nt // w
        cost = -(-ni // w) * w * (-(-nj // h) * h) * fac[w]
        if least is None or cost < least:
            best, least = w, cost
    return best


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
def test_forward_batch_per_field_tiles(batch, dtype):
    """Without a tile option each field runs its own tile shape in the same
    launch; every field equals its separate launch with that tile."""
    print(f"batched forward, per-field tiles, {dtype}", flush=True)
    api.stencil_clear_tuning()  # no tuned entries: the cost rule decides
    items = _items(batch, dtype)
    _run_batched(items, dtype)
    sep = _items(batch, dtype)
    shapes = set()
    for it in sep:
        ni, nj, nk = it["domain"]
        nt = 128 if dtype == torch.float64 and nk > 80 else 256
        tile = _least_cost_tile(ni, nj, nt, dtype)
        shapes.add(tile)
        o = api.Options(tile_i=tile)
        o.workspace = fields.workspace(api.OP_STEP, dtype, it["domain"], o)
        api.stencil_step(it["u"], it["data"], it["w"], it["out"], it["domain"], inputs.COEFF, inputs.DT_DZ,
                         mask=it["mask"], opts=o)
    torch.cuda.synchronize()
    assert len(shapes) > 1  # the workload mixes tile shapes in one launch
    for a, b in zip(items, sep):
        assert torch.equal(_interior(a), _interior(b)), a["domain"]
        assert torch.equal(a["mask"], b["mask"]), a["domain"]


def _adjoint_items(items, dtype, with_dbar):
    adj = []
    for n, it in enumerate(items):
        ni, nj, nk = it["domain"]
        st = _storage(ni, nj, nk)
        ob = inputs.cotangent(*st)
        adj.append(dict(x_bar=fields.from_interior(ob, dtype, DEV), w=it["w"], mask=it["mask"],
                        u_bar=fields.alloc(*st, dtype, DEV, fill=123.0),
                        data_bar=fields.alloc(*st, dtype, DEV, halo=0, fill=0.0) if with_dbar else None,
                        domain=it["domain"], coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, ob=ob))
    return adj


def _run_adjoint_batched(adj, dtype, tile=0):
    ws = _ws(api.stencil_batch_adjoint_workspace_bytes(dtype, adj))
    api.stencil_step_adjoint_batched(dtype, adj, ws, opts=api.Options(tile_i=tile))
    return ws


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("with_dbar", [True, False], ids=["dbar", "ws"])
def test_adjoint_batch_vs_oracle(batch, dtype, with_dbar):
    print(f"batched adjoint, 32 fields, dbar={with_dbar}, {dtype}", flush=True)
    items = _items(batch, dtype)
    _run_batched(items, dtype)
    adj = _adjoint_items(items, dtype, with_dbar)
    _run_adjoint_batched(adj, dtype)
    torch.cuda.synchronize()
    ref = _oracle_forward(batch, dtype)
    coeff = c_scalar(inputs.COEFF, dtype)
    for (ni, nj, nk, f), a, (_, mx, my) in zip(batch, adj, ref):
        r = _ref(f, dtype)
        ob = round_f32(a["ob"]) if dtype == torch.float32 else a["ob"]
        ubr, dbr = orc.step_adjoint(ob, r.w, mx, my, coeff, inputs.DT_DZ)
        assert rel_err(host(fields.padded(a["u_bar"], ni, nj, nk)), ubr) <= TOL[dtype], a["domain"]
        if with_dbar:
            assert rel_err(host(fields.interior(a["data_bar"], ni, nj, nk)), dbr) <= TOL[dtype], a["domain"]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("tile", [64, 16])
def test_adjoint_batch_vs_separate(batch, dtype, tile):
    print(f"batched adjoint vs separate launches, tile {tile}, {dtype}", flush=True)
    items = _items(batch, dtype)
    _run_batched(items, dtype)
    adj = _adjoint_items(items, dtype, True)
    _run_adjoint_batched(adj, dtype, tile)
    sep = _adjoint_items(items, dtype, True)
    for a in sep:
        o = api.Options(tile_i=tile)
        api.stencil_step_adjoint(a["x_bar"], a["w"], a["mask"], a["u_bar"], a["data_bar"], a["domain"],
                                 inputs.COEFF, inputs.DT_DZ, opts=o)
    torch.cuda.synchronize()
    for a, b in zip(adj, sep):
        ni, nj, nk = a["domain"]
        pa, pb = fields.padded(a["u_bar"], ni, nj, nk), fields.padded(b["u_bar"], ni, nj, nk)
        da, db = fields.interior(a["data_bar"], ni, nj, nk), fields.interior(b["data_bar"], ni, nj, nk)
        assert torch.equal(pa, pb) and torch.equal(da, db), a["domain"]


# ------------------------------------------------------------ small batches
SMALL = [(67, 45, 7), (1, 1, 1), (0, 12, 8), (33, 17, 144), (20, 9, 0), (130, 3, 2), (5, 70, 81),
         (64, 4, 97), (12, 0, 5)]


def _small_batch(seed):
    return [(ni, nj, nk, inputs.fields_sized(*_storage(ni, nj, nk), seed=seed + n))
            for n, (ni, nj, nk) in enumerate(SMALL)]


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
def test_small_batch_edges(dtype):
    """Empty fields in the batch, single points, the longest batched column,
    odd nk, and fields with and without a mask side by side."""
    print(f"batched edge cases {SMALL} {dtype}", flush=True)
    b = _small_batch(300)
    items = _items(b, dtype)
    for n in (1, 6):
        items[n]["mask"] = None
    _run_batched(items, dtype)
    torch.cuda.synchronize()
    coeff = c_scalar(inputs.COEFF, dtype)
    for (ni, nj, nk, f), it in zip(b, items):
        got = host(_interior(it))
        if ni * nj * nk == 0:
            assert np.all(got == 0.0)  # untouched
            continue
        r = _ref(f, dtype)
        nxt, mx, my = orc.step(r.u, r.data, r.w, coeff, inputs.DT_DZ, decide_f32=(dtype == torch.float32))
        assert rel_err(got, nxt[:, 2:-2, 2:-2]) <= TOL[dtype], (ni, nj, nk)
        if it["mask"] is not None:
            gx, gy = unpack_mask(it["mask"], ni, nj, nk)
            assert np.array_equal(gx, mx) and np.array_equal(gy, my), (ni, nj, nk)
    # the adjoint of the same batch (fields without a mask get the oracle's)
    for n in (1, 6):
        ni, nj, nk = SMALL[n]
        items[n]["mask"] = fields.mask_tensor(SMALL[n], DEV)
        o = api.Options()
        o.workspace = fields.workspace(api.OP_STEP, dtype, SMALL[n], o)
        it = items[n]
        api.stencil_step(it["u"], it["data"], it["w"], fields.alloc(ni, nj, nk, dtype, DEV), it["domain"],
                         inputs.COEFF, inputs.DT_DZ, mask=it["mask"], opts=o)
    adj = _adjoint_items(items, dtype, False)
    _run_adjoint_batched(adj, dtype)
    torch.cuda.synchronize()
    for (ni, nj, nk, f), a, it in zip(b, adj, items):
        if nk == 0:
            assert torch.all(a["u_bar"].tensor == 123.0)  # nothing to write
            continue
        r = _ref(f, dtype)
        ob = round_f32(a["ob"]) if dtype == torch.float32 else a["ob"]
        if ni * nj == 0:
            ubr = np.zeros((nk, nj + 4, ni + 4))
        else:
            mx, my = unpack_mask(it["mask"], ni, nj, nk)
            ubr, _ = orc.step_adjoint(ob, r.w, mx, my, coeff, inputs.DT_DZ)
        assert rel_err(host(fields.padded(a["u_bar"], ni, nj, nk)), ubr) <= TOL[dtype], (ni, nj, nk)


def test_repeat_and_graph_replay():
    """The work queue is rebuilt by every call: repeated calls and replays
    of a captured call give the eager result, with eager work in between."""
    dtype = torch.float64
    b = _small_batch(400)
    items = _items(b, dtype)
    ws = _ws(api.stencil_batch_workspace_bytes(dtype, items))
    api.stencil_step_batched(dtype, items, ws)
    torch.cuda.synchronize()
    first = [_interior(it).clone() for it in items]
    for it in items:
        it["out"].tensor.zero_()
    api.stencil_step_batched(dtype, items, ws)
    torch.cuda.synchronize()
    for it, ref in zip(items, first):
        assert torch.equal(_interior(it), ref)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        s.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            api.stencil_step_batched(dtype, items, ws, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:
            it["out"].tensor.fill_(float(rep))
        api.stencil_step_batched(dtype, items[:2], ws)  # other eager use of the workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, ref in zip(items, first):
            assert torch.equal(_interior(it), ref), (rep, it["domain"])
