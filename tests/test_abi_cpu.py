"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every declared entry point, and argument validation rejects bad
calls with the documented status codes before any device work.  Field data
pointers here are fake (never dereferenced: validation reads metadata only).
"""
import ctypes
import json
import os
import re

import pytest

from paper_2311_08322_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), f"{n} declared in stencil.h but not exported"
    # and the binding covers the same names
    from paper_2311_08322_amd import api

    for n in names:
        assert hasattr(api, n), f"python binding lacks {n}"


def test_version_and_limits(L):
    assert L.stencil_version() == 3
    assert L.stencil_max_fused_nk(1) >= 137


def test_mask_bytes(L):
    # 64x64x16: one word per row; X and Y planes 8*64*16 B; edges 64*16 B each
    assert L.stencil_mask_bytes(_lib.domain3((64, 64, 16))) == 8192 * 2 + 1024 * 2
    # 65 columns need two words per row
    d = (65, 3, 2)
    plane = (8 * 2 * 3 * 2 + 255) // 256 * 256
    assert L.stencil_mask_bytes(_lib.domain3(d)) == 2 * plane + 256 + 256
    assert L.stencil_mask_bytes(_lib.domain3((-1, 3, 2))) == 0
    assert L.stencil_mask_bytes(None) == 0
    assert L.stencil_mask_bytes(_lib.domain3((0, 5, 5))) == 0


def test_workspace_bytes(L):
    d = _lib.domain3((64, 48, 16))
    assert L.stencil_workspace_bytes(_lib.OP_STEP, _lib.F64, d, None) == 0
    o = _lib.StencilOptions()
    o.impl = _lib.IMPL_PLAIN
    plain = L.stencil_workspace_bytes(_lib.OP_STEP, _lib.F64, d, ctypes.byref(o))
    # lap, fx, fy and the two elimination arrays: about 5 fields
    n = 64 * 48 * 16 * 8
    assert 5 * n <= plain <= 5 * n + 5 * 256 + 8 * (66 * 50 - 64 * 48) * 16 + 8 * (65 + 49) * 16
    assert L.stencil_workspace_bytes(_lib.OP_STEP, _lib.F32, d, ctypes.byref(o)) < plain
    # the step adjoint keeps lambda in the workspace when data_bar is absent
    assert L.stencil_workspace_bytes(_lib.OP_STEP_ADJOINT, _lib.F64, d, None) >= n
    # columns longer than the fused classes need the plain workspace
    long = _lib.domain3((8, 8, 200))
    assert L.stencil_workspace_bytes(_lib.OP_STEP, _lib.F64, long, None) > 0


# ----------------------------------------------------------------- validation
BASE = 0x7F0000000000


def fld(ni, nj, nk, halo=2, kextra=0, base=BASE, es=8):
    f = _lib.StencilField()
    f.data = base
    Ni, Nj = ni + 2 * halo, nj + 2 * halo
    f.shape = _lib.I64x3(Ni, Nj, nk + kextra)
    f.stride = _lib.I64x3(1, Ni, Ni * Nj)
    f.origin = _lib.I64x3(halo, halo, 0)
    return f


def fields(ni=16, nj=12, nk=8):
    span = (ni + 4) * (nj + 4) * (nk + 1) * 8 + 4096
    u = fld(ni, nj, nk, base=BASE)
    data = fld(ni, nj, nk, halo=0, base=BASE + span)
    w = fld(ni, nj, nk, halo=0, kextra=1, base=BASE + 2 * span)
    out = fld(ni, nj, nk, base=BASE + 3 * span)
    return u, data, w, out, _lib.domain3((ni, nj, nk))


def step(L, u, data, w, out, d, mask=None, opts=None, dt=_lib.F64):
    b = ctypes.byref
    return L.stencil_step(dt, b(u) if u else None, b(data), b(w), b(out), d, 0.025, 0.5, mask,
                          b(opts) if opts else None, None)


def code(name):
    return _lib.CODES[name]


def test_null_and_dtype(L):
    u, data, w, out, d = fields()
    assert step(L, None, data, w, out, d) == code("STENCIL_E_NULL")
    assert "u" in _lib.last_error()
    for dt in (7, -1, 2, -2147483648, 2147483647):  # every 32-bit value is a valid argument
        assert step(L, u, data, w, out, d, dt=dt) == code("STENCIL_E_DTYPE")
    u.data = None
    assert step(L, u, data, w, out, d) == code("STENCIL_E_NULL")
    u, data, w, out, d = fields()
    u.data = BASE + 4  # not 8-byte aligned for FP64
    assert step(L, u, data, w, out, d) == code("STENCIL_E_DTYPE")


def test_halo_and_shape(L):
    u, data, w, out, d = fields()
    u.origin = _lib.I64x3(1, 2, 0)
    assert step(L, u, data, w, out, d) == code("STENCIL_E_HALO")
    u, data, w, out, d = fields()
    u.shape = _lib.I64x3(u.shape[0] - 1, u.shape[1], u.shape[2])
    assert step(L, u, data, w, out, d) == code("STENCIL_E_HALO")
    u, data, w, out, d = fields()
    w.shape = _lib.I64x3(w.shape[0], w.shape[1], w.shape[2] - 1)  # nk levels, needs nk+1
    assert step(L, u, data, w, out, d) == code("STENCIL_E_SHAPE")
    assert "w" in _lib.last_error()
    u, data, w, out, d = fields()
    d2 = _lib.domain3((16, 13, 8))
    assert step(L, u, data, w, out, d2) in (code("STENCIL_E_HALO"), code("STENCIL_E_SHAPE"))
    assert step(L, u, data, w, out, _lib.domain3((16, -1, 8))) == code("STENCIL_E_SHAPE")


def test_strides(L):
    u, data, w, out, d = fields()
    u.stride = _lib.I64x3(2, u.stride[1], u.stride[2])
    assert step(L, u, data, w, out, d) == code("STENCIL_E_STRIDE")
    u, data, w, out, d = fields()
    u.stride = _lib.I64x3(1, u.shape[0] - 1, u.stride[2])
    assert step(L, u, data, w, out, d) == code("STENCIL_E_STRIDE")


def test_level_window_limit(L):
    # kernels predicate a lane's access off with the byte offset 0xFFFFFFF0,
    # which must lie outside every level window: an FP32 output one point
    # wide whose level spans 0xFFFFFFF0 bytes (below 4 GiB) is refused
    u, data, w, out, d = fields(ni=1, nj=1, nk=1)
    rows = (0xFFFFFFF0 // 4 - 5) // 5
    assert (5 * rows + 5) * 4 == 0xFFFFFFF0
    out = _lib.StencilField()
    out.data = BASE + (1 << 36)
    out.shape = _lib.I64x3(5, rows, 1)
    out.stride = _lib.I64x3(1, 5, 5 * rows)
    out.origin = _lib.I64x3(2, 2, 0)
    assert step(L, u, data, w, out, d, dt=_lib.F32) == code("STENCIL_E_UNSUPPORTED")
    assert "window" in _lib.last_error()
    # 16 bytes less passes that check (and fails a later one: an origin that
    # puts the domain past the field's end)
    out.shape = _lib.I64x3(5, rows - 1, 1)
    out.stride = _lib.I64x3(1, 5, 5 * rows)
    assert (5 * (rows - 1) + 5) * 4 <= 0xFFFFFFF0 - 16
    out.origin = _lib.I64x3(5, 2, 0)
    assert step(L, u, data, w, out, d, dt=_lib.F32) in (code("STENCIL_E_HALO"), code("STENCIL_E_SHAPE"))
    assert "window" not in _lib.last_error()


def test_alias(L):
    u, data, w, out, d = fields()
    out.data = u.data  # in-place is forbidden (whole-domain assignment semantics)
    assert step(L, u, data, w, out, d) == code("STENCIL_E_ALIAS")
    u, data, w, out, d = fields()
    out.data = data.data + 8 * 5
    assert step(L, u, data, w, out, d) == code("STENCIL_E_ALIAS")
    u, data, w, out, d = fields()
    mask = out.data + 8  # mask overlapping the output
    assert step(L, u, data, w, out, d, mask=mask) == code("STENCIL_E_ALIAS")


def test_options(L):
    u, data, w, out, d = fields()
    o = _lib.StencilOptions()
    o.impl = 9
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
    o = _lib.StencilOptions()
    o.tile_i, o.tile_j = 48, 4
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
    o.tile_i, o.tile_j = 64, 8  # neither 256 nor 128 columns
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
    # 128-column tiles run the two-ended step only
    for ti, tj in ((64, 2), (32, 4), (16, 8)):
        o = _lib.StencilOptions()
        o.tile_i, o.tile_j, o.column_store = ti, tj, _lib.COLUMN_REGISTERS
        assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_UNSUPPORTED")
        assert "two-ended" in _lib.last_error()
        o.column_store = _lib.COLUMN_SPLIT  # accepted: fails later, at the device check
        assert step(L, u, data, w, out, d, opts=o) not in (code("STENCIL_E_ARG"), code("STENCIL_E_UNSUPPORTED"))
    o = _lib.StencilOptions()
    o.impl = _lib.IMPL_PLAIN  # no workspace
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_WORKSPACE")
    o.workspace = 0x7E0000000000
    o.workspace_bytes = 64
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_WORKSPACE")
    assert "smaller" in _lib.last_error()


def test_long_columns_need_plain(L):
    u, data, w, out, d = fields(8, 8, 200)
    o = _lib.StencilOptions()
    o.impl = _lib.IMPL_FUSED
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_UNSUPPORTED")
    # AUTO falls back to PLAIN, which then wants its workspace
    assert step(L, u, data, w, out, d) == code("STENCIL_E_WORKSPACE")


def test_empty_domain_is_a_noop(L):
    u, data, w, out, d = fields(16, 12, 8)
    assert step(L, u, data, w, out, _lib.domain3((0, 12, 8))) == 0
    assert step(L, u, data, w, out, _lib.domain3((16, 12, 0))) == 0


def test_adjoint_validation(L):
    b = ctypes.byref
    u, data, w, out, d = fields()
    xb = fld(16, 12, 8, halo=0, base=BASE + (1 << 30))
    ub = fld(16, 12, 8, base=BASE + (2 << 30))
    # u_bar needs the halo (it is written there)
    ub2 = fld(16, 12, 8, halo=0, base=BASE + (2 << 30))
    assert L.stencil_step_adjoint(1, b(xb), b(w), BASE + (3 << 30), b(ub2), None, d, 0.025, 0.5, None,
                                  None) == code("STENCIL_E_HALO")
    # missing mask
    assert L.stencil_step_adjoint(1, b(xb), b(w), None, b(ub), b(data), d, 0.025, 0.5, None,
                                  None) == code("STENCIL_E_NULL")
    # data_bar aliasing x_bar
    assert L.stencil_step_adjoint(1, b(xb), b(w), BASE + (3 << 30), b(ub), b(xb), d, 0.025, 0.5, None,
                                  None) == code("STENCIL_E_ALIAS")
    # no data_bar and no workspace for lambda
    assert L.stencil_step_adjoint(1, b(xb), b(w), BASE + (3 << 30), b(ub), None, d, 0.025, 0.5, None,
                                  None) == code("STENCIL_E_WORKSPACE")
    assert L.stencil_hdiff_adjoint(1, b(xb), None, b(ub), d, 0.025, None, None) == code("STENCIL_E_NULL")
    assert L.stencil_vadv_adjoint(1, b(xb), b(w), b(xb), d, 0.5, None, None) == code("STENCIL_E_ALIAS")


def test_graph_capture_validation(L):
    b = ctypes.byref
    u, data, w, out, d = fields()
    h = ctypes.c_void_p()
    assert L.stencil_graph_capture_steps(1, 0, b(u), b(out), b(data), b(w), d, 0.025, 0.5, None,
                                         0x1234, b(h)) == code("STENCIL_E_ARG")
    assert L.stencil_graph_capture_steps(1, 4, b(u), b(out), b(data), b(w), d, 0.025, 0.5, None,
                                         None, b(h)) == code("STENCIL_E_ARG")
    assert L.stencil_graph_capture_steps(1, 4, b(u), b(u), b(data), b(w), d, 0.025, 0.5, None,
                                         0x1234, b(h)) == code("STENCIL_E_ALIAS")
    assert L.stencil_graph_launch(None, None) == code("STENCIL_E_NULL")
    assert L.stencil_graph_destroy(None) == 0


# ----------------------------------------------------------------- tuning table
def test_tuning_json_roundtrip(L, tmp_path):
    assert L.stencil_clear_tuning() == 0
    d = _lib.domain3((256, 256, 80))
    ti, tj, col, order = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()

    def look(dom):
        return L.stencil_tuning_lookup(1, _lib.OP_STEP, dom, ctypes.byref(ti), ctypes.byref(tj), ctypes.byref(col),
                                       ctypes.byref(order))

    assert look(d) == 0
    assert (ti.value, tj.value, order.value) == (64, 4, _lib.ORDER_XCD)
    # the order output may be NULL
    assert L.stencil_tuning_lookup(1, _lib.OP_STEP, d, ctypes.byref(ti), ctypes.byref(tj), ctypes.byref(col),
                                   None) == 0
    p = tmp_path / "tune.json"
    doc = {"arch": "gfx950", "version": 1, "entries": [
        {"dtype": 1, "op": _lib.OP_STEP, "nk_class": 5, "area_class": 2, "tile_i": 32, "tile_j": 8,
         "column_store": 2, "us": 12.5}]}
    p.write_text(json.dumps(doc))
    assert L.stencil_load_tuning(str(p).encode()) == 0
    assert look(d) == 0
    # an entry without a tile order (an older table) takes the XCD runs
    assert (ti.value, tj.value, col.value, order.value) == (32, 8, 2, _lib.ORDER_XCD)
    # another size class is untouched
    d2 = _lib.domain3((64, 64, 16))
    assert look(d2) == 0
    assert ti.value == 64
    doc["entries"][0]["tile_order"] = _lib.ORDER_DISPATCH
    doc["entries"][0]["column_store"] = 3
    p.write_text(json.dumps(doc))
    assert L.stencil_load_tuning(str(p).encode()) == 0
    assert look(d) == 0 and (col.value, order.value) == (3, _lib.ORDER_DISPATCH)
    q = tmp_path / "saved.json"
    assert L.stencil_save_tuning(str(q).encode()) == 0
    saved = json.loads(q.read_text())
    assert saved["arch"] == "gfx950" and len(saved["entries"]) == 1
    assert saved["entries"][0]["tile_i"] == 32 and saved["entries"][0]["tile_order"] == _lib.ORDER_DISPATCH
    assert L.stencil_clear_tuning() == 0
    assert L.stencil_load_tuning(str(q).encode()) == 0
    assert look(d) == 0
    assert ti.value == 32 and order.value == _lib.ORDER_DISPATCH
    bad = tmp_path / "bad.json"
    bad.write_text('{"arch": "gfx950", "entries": [{"dtype": 1, "op": 2, "tile_i": 48}]}')
    assert L.stencil_load_tuning(str(bad).encode()) == code("STENCIL_E_ARG")
    doc["entries"][0]["tile_order"] = 7
    bad.write_text(json.dumps(doc))
    assert L.stencil_load_tuning(str(bad).encode()) == code("STENCIL_E_ARG")
    # a 128-column tile is a two-ended step entry only
    doc["entries"][0].update(tile_order=_lib.ORDER_XCD, tile_i=32, tile_j=4, column_store=3)
    p.write_text(json.dumps(doc))
    assert L.stencil_load_tuning(str(p).encode()) == 0
    assert look(d) == 0 and (ti.value, tj.value, col.value) == (32, 4, 3)
    doc["entries"][0]["column_store"] = 1
    bad.write_text(json.dumps(doc))
    assert L.stencil_load_tuning(str(bad).encode()) == code("STENCIL_E_ARG")
    assert L.stencil_load_tuning(b"/nonexistent/x.json") == code("STENCIL_E_ARG")
    assert L.stencil_clear_tuning() == 0


def test_binding_refuses_unknown_dtype():
    import torch

    from paper_2311_08322_amd import api

    t = torch.zeros((2, 8, 8), dtype=torch.int32)
    with pytest.raises(api.StencilError):
        api.stencil_hdiff(api.Field(t, (2, 2, 0)), api.Field(t.clone(), (2, 2, 0)), (4, 4, 2), 0.025,
                          stream=0)


# ----------------------------------------------------------------- batched
def batch_items(sizes, base=BASE):
    arr = (_lib.StencilBatchItem * len(sizes))()
    for n, (ni, nj, nk) in enumerate(sizes):
        u, data, w, out, d = fields(ni, nj, nk)
        off = base + n * (1 << 32)  # each item in its own 4 GiB window
        for f in (u, data, w, out):
            f.data = f.data - BASE + off
        arr[n].u, arr[n].data, arr[n].w, arr[n].out = u, data, w, out
        arr[n].domain = _lib.I64x3(ni, nj, nk)
        arr[n].coeff, arr[n].dt_dz = 0.025, 0.5
    return arr


def test_batch_validation(L):
    items = batch_items([(16, 12, 8), (20, 9, 30)])
    need = L.stencil_batch_workspace_bytes(1, 2, items)
    assert need > 0 and need % 256 == 0
    ws = BASE + (64 << 32)
    run = lambda arr, n=2, ws=ws, nb=need, o=None: L.stencil_step_batched(  # noqa: E731
        1, n, arr, ws, nb, ctypes.byref(o) if o else None, None)
    assert run(items, nb=need - 1) == code("STENCIL_E_WORKSPACE")
    assert run(items, ws=None) == code("STENCIL_E_WORKSPACE")
    assert run(items, ws=ws + 8) == code("STENCIL_E_WORKSPACE")  # the table wants 256-B alignment
    assert run(items, n=-1) == code("STENCIL_E_ARG")
    assert run(None, n=2) == code("STENCIL_E_NULL")
    o = _lib.StencilOptions()
    o.impl = _lib.IMPL_PLAIN
    assert run(items, o=o) == code("STENCIL_E_UNSUPPORTED")
    # the workspace may not overlap any field
    assert run(items, ws=items[1].u.data) == code("STENCIL_E_ALIAS")
    # one item's output may not touch another item's buffers (all run at once)
    bad = batch_items([(16, 12, 8), (20, 9, 30)])
    bad[1].out.data = bad[0].u.data
    assert run(bad) == code("STENCIL_E_ALIAS")
    assert "item 1" in _lib.last_error() and "item 0" in _lib.last_error()
    bad = batch_items([(16, 12, 8), (20, 9, 30)])
    bad[0].mask = bad[1].w.data
    assert run(bad) == code("STENCIL_E_ALIAS")
    # per-item rules name the item
    bad = batch_items([(16, 12, 8), (20, 9, 30)])
    bad[1].u.origin = _lib.I64x3(1, 2, 0)
    assert run(bad) == code("STENCIL_E_HALO")
    assert _lib.last_error().startswith("item 1")
    # columns longer than the batched classes
    long = batch_items([(16, 12, 8), (8, 8, 145)])
    assert run(long, nb=L.stencil_batch_workspace_bytes(1, 2, long)) == code("STENCIL_E_UNSUPPORTED")
    # a batch with no interior work is a no-op that needs no workspace (and no device)
    empty = batch_items([(0, 12, 8), (20, 9, 0)])
    assert L.stencil_batch_workspace_bytes(1, 2, empty) == 0
    assert run(empty, ws=None, nb=0) == 0
    assert L.stencil_step_batched(1, 0, None, None, 0, None, None) == 0


def test_batch_noalloc_validation(L):
    """The no-allocation batch validates as stencil_step_batched does and
    refuses a work list larger than its fixed array before any device work."""
    m = re.search(r"#define\s+STENCIL_NOALLOC_SCRATCH_BYTES\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == _lib.NOALLOC_SCRATCH_BYTES
    run = lambda arr, n=2, o=None: L.stencil_step_batched_noalloc(  # noqa: E731
        1, n, arr, ctypes.byref(o) if o else None, None)
    items = batch_items([(16, 12, 8), (20, 9, 30)])
    assert run(items, n=-1) == code("STENCIL_E_ARG")
    assert run(None, n=2) == code("STENCIL_E_NULL")
    o = _lib.StencilOptions()
    o.impl = _lib.IMPL_PLAIN
    assert run(items, o=o) == code("STENCIL_E_UNSUPPORTED")
    bad = batch_items([(16, 12, 8), (20, 9, 30)])
    bad[1].out.data = bad[0].u.data
    assert run(bad) == code("STENCIL_E_ALIAS")
    long = batch_items([(16, 12, 8), (8, 8, 145)])
    assert run(long) == code("STENCIL_E_UNSUPPORTED")
    # any batch of up to 256 fields fits the array (both FP64 column groups
    # present, the worst case of the table layout) ...
    sizes = [(16, 12, 8 if n % 2 else 120) for n in range(256)]
    many = batch_items(sizes)
    for dt in (_lib.F32, _lib.F64):
        assert 0 < L.stencil_batch_workspace_bytes(dt, 256, many) <= _lib.NOALLOC_SCRATCH_BYTES
    # ... and a longer one is refused, naming the limit
    more = batch_items([(16, 12, 8)] * 300)
    assert L.stencil_batch_workspace_bytes(1, 300, more) > _lib.NOALLOC_SCRATCH_BYTES
    assert run(more, n=300) == code("STENCIL_E_UNSUPPORTED")
    assert str(_lib.NOALLOC_SCRATCH_BYTES) in _lib.last_error()
    # no work: a no-op without a device
    empty = batch_items([(0, 12, 8), (20, 9, 0)])
    assert run(empty) == 0
    assert L.stencil_step_batched_noalloc(1, 0, None, None, None) == 0


def test_batch_adjoint_workspace_and_validation(L):
    fw = batch_items([(16, 12, 8), (20, 9, 30)])
    arr = (_lib.StencilBatchAdjointItem * 2)()
    for n in range(2):
        arr[n].x_bar, arr[n].w, arr[n].u_bar = fw[n].data, fw[n].w, fw[n].u
        arr[n].domain, arr[n].coeff, arr[n].dt_dz = fw[n].domain, 0.025, 0.5
        arr[n].mask = fw[n].out.data  # distinct memory standing in for a mask
    without = L.stencil_batch_adjoint_workspace_bytes(1, 2, arr)
    # lambda of both items lives in the workspace when data_bar is absent
    assert without >= 8 * (16 * 12 * 8 + 20 * 9 * 30)
    arr[0].data_bar = fld(16, 12, 8, halo=0, base=BASE + (40 << 32))
    assert without - L.stencil_batch_adjoint_workspace_bytes(1, 2, arr) >= 8 * 16 * 12 * 8
    ws = BASE + (64 << 32)
    need = L.stencil_batch_adjoint_workspace_bytes(1, 2, arr)
    arr[1].mask = None
    assert L.stencil_step_adjoint_batched(1, 2, arr, ws, need, None, None) == code("STENCIL_E_NULL")
    arr[1].mask = fw[1].out.data
    arr[1].u_bar = fld(20, 9, 30, base=fw[0].u.data)  # two items writing one buffer
    assert L.stencil_step_adjoint_batched(1, 2, arr, ws, need, None, None) == code("STENCIL_E_ALIAS")


def test_param_adjoint_validation(L):
    b = ctypes.byref
    u, data, w, out, d = fields(16, 12, 8)
    lam = fld(16, 12, 8, halo=0, base=BASE + (5 << 32))
    x = fld(16, 12, 8, halo=0, base=BASE + (6 << 32))
    wb = fld(16, 12, 8, halo=0, kextra=1, base=BASE + (7 << 32))
    cb = BASE + (8 << 32)
    ws = BASE + (9 << 32)
    need = L.stencil_param_workspace_bytes(1, d)
    assert need >= 8 * 1 * 3 and need % 256 == 0  # one double per 64 x 4 tile
    call = lambda wbar=b(wb), coeff_bar=cb, ws=ws, nb=need: L.stencil_step_param_adjoint(  # noqa: E731
        1, b(u), b(w), b(x), b(lam), wbar, coeff_bar, d, 0.5, None, ws, nb, None)
    assert call(wbar=None, coeff_bar=None) == code("STENCIL_E_NULL")
    assert call(ws=None) == code("STENCIL_E_WORKSPACE")
    assert call(nb=need - 8) == code("STENCIL_E_WORKSPACE")
    assert call(coeff_bar=cb + 4) == code("STENCIL_E_DTYPE")
    assert call(coeff_bar=lam.data) == code("STENCIL_E_ALIAS")  # output inside an input
    assert call(ws=x.data) == code("STENCIL_E_ALIAS")
    wb2 = fld(16, 12, 8, halo=0, kextra=1, base=x.data)
    assert call(wbar=b(wb2)) == code("STENCIL_E_ALIAS")
    short = fld(16, 12, 8, halo=0, base=BASE + (7 << 32))  # nk levels, w_bar needs nk + 1
    assert call(wbar=b(short)) == code("STENCIL_E_SHAPE")
    # w_bar alone needs no workspace
    assert L.stencil_param_workspace_bytes(1, _lib.domain3((0, 12, 8))) == 0


def test_boundary_option_and_halo_update_validation(L):
    u, data, w, out, d = fields()
    o = _lib.StencilOptions()
    o.boundary = 7
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
    o.boundary = _lib.BOUNDARY_PERIODIC
    out0 = fld(16, 12, 8, halo=0, base=out.data)  # a periodic step writes out's halo
    assert step(L, u, data, w, out0, d, opts=o) == code("STENCIL_E_HALO")
    b = ctypes.byref
    assert L.stencil_halo_update(1, b(out0), d, 1, None) == code("STENCIL_E_HALO")
    assert L.stencil_halo_update(1, b(u), d, 5, None) == code("STENCIL_E_ARG")
    assert L.stencil_halo_update(1, b(u), d, 0, None) == 0  # frozen: nothing to do
    assert L.stencil_halo_update(1, b(u), _lib.domain3((0, 12, 8)), 1, None) == 0
    items = batch_items([(16, 12, 8)])
    assert L.stencil_step_batched(1, 1, items, BASE + (64 << 32), 1 << 20, b(o), None) == code(
        "STENCIL_E_UNSUPPORTED")


def test_autotune_fields_validation(L):
    """Tuning on caller fields: only the step, the step's field rules, no
    output overlapping an input -- all refused before any device work."""
    b = ctypes.byref
    u, data, w, out, d = fields()
    us = ctypes.c_double()
    assert L.stencil_autotune_fields(1, _lib.OP_HDIFF, b(u), b(data), b(w), b(out), d, 2, None, b(us)) == code(
        "STENCIL_E_ARG")
    assert L.stencil_autotune_fields(1, _lib.OP_STEP, b(u), b(data), b(w), b(u), d, 2, None, b(us)) == code(
        "STENCIL_E_ALIAS")
    assert L.stencil_autotune_fields(1, _lib.OP_STEP, None, b(data), b(w), b(out), d, 2, None, b(us)) == code(
        "STENCIL_E_NULL")
    assert L.stencil_autotune_fields(7, _lib.OP_STEP, b(u), b(data), b(w), b(out), d, 2, None, b(us)) == code(
        "STENCIL_E_DTYPE")
    assert L.stencil_autotune_fields(1, _lib.OP_STEP, b(u), b(data), b(w), b(out), _lib.domain3((0, 4, 4)), 2,
                                     None, b(us)) == code("STENCIL_E_SHAPE")


def test_tile_order_validation(L):
    """An unknown tile order is refused before any device work."""
    u, data, w, out, d = fields()
    o = _lib.StencilOptions()
    for bad in (-1, 3):
        o.tile_order = bad
        assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
        assert "tile_order" in _lib.last_error()


def test_generalised_diffusion_validation(L):
    """hdiff_form and coeff_field: unknown forms, coefficient fields of the
    wrong size or overlapping an output, and the forms without a kernel
    (PLAIN, long columns, batched) are refused before any device work."""
    b = ctypes.byref
    u, data, w, out, d = fields()
    o = _lib.StencilOptions()
    o.hdiff_form = 3
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_ARG")
    o.hdiff_form = _lib.HDIFF_DAMPING
    o.impl = _lib.IMPL_PLAIN
    o.workspace = BASE + (40 << 32)
    o.workspace_bytes = 1 << 30
    assert step(L, u, data, w, out, d, opts=o) == code("STENCIL_E_UNSUPPORTED")
    assert L.stencil_hdiff(1, b(u), b(out), d, 0.025, None, b(o), None) == code("STENCIL_E_UNSUPPORTED")
    o = _lib.StencilOptions()
    o.hdiff_form = _lib.HDIFF_DAMPING
    lu, ldata, lw, lout, ld = fields(16, 12, 145)
    assert step(L, lu, ldata, lw, lout, ld, opts=o) == code("STENCIL_E_UNSUPPORTED")  # FP64 nk > 144
    kap = fld(16, 12, 8, halo=0, base=BASE + (41 << 32))
    o.coeff_field = ctypes.pointer(kap)
    small = fld(15, 12, 8, halo=0, base=BASE + (41 << 32))
    o2 = _lib.StencilOptions()
    o2.coeff_field = ctypes.pointer(small)
    assert step(L, u, data, w, out, d, opts=o2) == code("STENCIL_E_SHAPE")
    inside = fld(16, 12, 8, halo=0, base=out.data)
    o3 = _lib.StencilOptions()
    o3.coeff_field = ctypes.pointer(inside)
    assert step(L, u, data, w, out, d, opts=o3) == code("STENCIL_E_ALIAS")
    assert L.stencil_hdiff(1, b(u), b(out), d, 0.025, None, b(o3), None) == code("STENCIL_E_ALIAS")
    ub = fld(16, 12, 8, base=out.data)
    assert L.stencil_hdiff_adjoint(1, b(data), BASE + (42 << 32), b(ub), d, 0.025, b(o3), None) == code(
        "STENCIL_E_ALIAS")
    items = batch_items([(16, 12, 8)])
    assert L.stencil_step_batched(1, 1, items, BASE + (64 << 32), 1 << 20, b(o), None) == code(
        "STENCIL_E_UNSUPPORTED")
    # the parameter adjoint: no scalar coeff_bar for a coefficient field
    lam = fld(16, 12, 8, halo=0, base=BASE + (5 << 32))
    x = fld(16, 12, 8, halo=0, base=BASE + (6 << 32))
    wb = fld(16, 12, 8, halo=0, kextra=1, base=BASE + (7 << 32))
    ws = BASE + (9 << 32)
    need = L.stencil_param_workspace_bytes(1, d)
    assert L.stencil_step_param_adjoint(1, b(u), b(w), b(x), b(lam), b(wb), BASE + (8 << 32), d, 0.5, b(o),
                                        ws, need, None) == code("STENCIL_E_ARG")
    # the coefficient-field gradient
    kb = fld(16, 12, 8, halo=0, base=BASE + (43 << 32))
    assert L.stencil_coeff_field_adjoint(1, b(u), b(lam), None, d, None, None) == code("STENCIL_E_NULL")
    kb_in = fld(16, 12, 8, halo=0, base=lam.data)
    assert L.stencil_coeff_field_adjoint(1, b(u), b(lam), b(kb_in), d, None, None) == code("STENCIL_E_ALIAS")
    kb_short = fld(16, 12, 7, halo=0, base=BASE + (43 << 32))
    assert L.stencil_coeff_field_adjoint(1, b(u), b(lam), b(kb_short), d, None, None) == code("STENCIL_E_SHAPE")
    assert L.stencil_coeff_field_adjoint(1, b(u), b(lam), b(kb), _lib.domain3((0, 12, 8)), None, None) == 0
    bad = _lib.StencilOptions()
    bad.hdiff_form = -1
    assert L.stencil_coeff_field_adjoint(1, b(u), b(lam), b(kb), d, b(bad), None) == code("STENCIL_E_ARG")


def test_field_descriptor_follows_the_tensor():
    """The binding keeps a field's C descriptor between calls and rebuilds it
    whenever the storage, shape, strides or origin change."""
    import torch

    from paper_2311_08322_amd import api
    t = torch.zeros((3, 8, 10), dtype=torch.float64)
    f = api.Field(t, (2, 2, 0))
    a = f.c()
    assert f.c() is a  # unchanged: the same descriptor
    assert (a.data, list(a.shape), list(a.stride), list(a.origin)) == (t.data_ptr(), [10, 8, 3], [1, 10, 80], [2, 2, 0])
    f.origin = (3, 2, 1)
    assert list(f.c().origin) == [3, 2, 1]
    u = torch.zeros((3, 8, 12), dtype=torch.float64)[:, :, 1:11]
    f.tensor = u
    b = f.c()
    assert (b.data, list(b.shape), list(b.stride)) == (u.data_ptr(), [10, 8, 3], [1, 12, 96])
    t2 = torch.zeros((3, 8, 10), dtype=torch.float64)
    f.tensor = t2
    t2.resize_(4, 9, 10)  # the same tensor object, new storage and shape
    c = f.c()
    assert (c.data, list(c.shape), list(c.stride)) == (t2.data_ptr(), [10, 9, 4], [1, 10, 90])
