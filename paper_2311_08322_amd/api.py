"""Python binding of the C ABI, one function per ``extern "C"`` entry point
(same names as ``include/stencil.h``).  Argument marshalling only: every step
of the stencils runs in the HIP kernels of ``libgt4mi.so``.

Fields are :class:`Field` objects: a torch tensor laid out (k, j, i) with
unit stride along i, plus the origin -- the (i, j, k) index of the tensor
element that is compute-domain point (0, 0, 0).  Masks and workspaces are
torch ``uint8`` device tensors (or ``None``).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import (BOUNDARY_FROZEN, BOUNDARY_PERIODIC, HDIFF_DAMPING, HDIFF_STATED, COLUMN_AUTO, COLUMN_OUTBUF, COLUMN_REGISTERS, COLUMN_SPLIT, F32, F64, IMPL_AUTO, IMPL_FUSED,
                   IMPL_PLAIN, OP_HDIFF, OP_HDIFF_ADJOINT, OP_STEP, OP_STEP_ADJOINT, OP_VADV,
                   OP_VADV_ADJOINT, ORDER_AUTO, ORDER_DISPATCH, ORDER_XCD, StencilError)

__all__ = [
    "Field", "Options", "StencilError", "F32", "F64",
    "IMPL_AUTO", "IMPL_FUSED", "IMPL_PLAIN", "ORDER_AUTO", "ORDER_XCD", "ORDER_DISPATCH", "BOUNDARY_FROZEN", "BOUNDARY_PERIODIC", "HDIFF_STATED", "HDIFF_DAMPING", "COLUMN_AUTO", "COLUMN_REGISTERS", "COLUMN_OUTBUF", "COLUMN_SPLIT",
    "OP_HDIFF", "OP_VADV", "OP_STEP", "OP_HDIFF_ADJOINT", "OP_VADV_ADJOINT", "OP_STEP_ADJOINT",
    "stencil_version", "stencil_last_error", "stencil_max_fused_nk", "stencil_mask_bytes",
    "stencil_workspace_bytes", "stencil_hdiff", "stencil_vadv", "stencil_step",
    "stencil_hdiff_adjoint", "stencil_vadv_adjoint", "stencil_step_adjoint",
    "stencil_param_workspace_bytes", "stencil_step_param_adjoint", "stencil_coeff_field_adjoint",
    "stencil_halo_update",
    "stencil_batch_workspace_bytes", "stencil_batch_adjoint_workspace_bytes",
    "stencil_step_batched", "stencil_step_adjoint_batched", "stencil_graph_capture_steps",
    "stencil_graph_launch", "stencil_graph_destroy", "stencil_autotune", "stencil_autotune_fields",
    "stencil_tuning_lookup",
    "stencil_save_tuning", "stencil_load_tuning", "stencil_clear_tuning",
]


@dataclass
class Field:
    tensor: torch.Tensor
    origin: Sequence[int] = (0, 0, 0)

    def c(self) -> _lib.StencilField:
        """The C descriptor, rebuilt only when the tensor's storage, shape,
        strides or the origin changed (building it costs a few microseconds
        per field, a noticeable part of a call on a small domain)."""
        t = self.tensor
        key = (t.data_ptr(), t.shape, t.stride(), tuple(self.origin))
        cached = self.__dict__.get("_c")
        if cached is not None and cached[0] == key:
            return cached[1]
        if t.dim() != 3:
            raise ValueError("a field tensor is 3-D, laid out (k, j, i)")
        f = _lib.StencilField()
        f.data = key[0]
        f.shape = _lib.I64x3(t.shape[2], t.shape[1], t.shape[0])
        f.stride = _lib.I64x3(t.stride(2), t.stride(1), t.stride(0))
        f.origin = _lib.I64x3(*[int(x) for x in self.origin])
        self.__dict__["_c"] = (key, f)
        return f

    @property
    def dtype(self):
        return self.tensor.dtype


@dataclass
class Options:
    impl: int = IMPL_AUTO
    tile_i: int = 0
    tile_j: int = 0
    column_store: int = COLUMN_AUTO
    workspace: Optional[torch.Tensor] = None
    boundary: int = BOUNDARY_FROZEN
    hdiff_form: int = HDIFF_STATED
    coeff_field: Optional["Field"] = None  # per-point coefficient (interior layout)
    tile_order: int = ORDER_AUTO

    def c(self) -> _lib.StencilOptions:
        o = _lib.StencilOptions()
        o.impl = self.impl
        o.tile_i = self.tile_i
        o.tile_j = self.tile_j
        o.column_store = self.column_store
        if self.workspace is not None:
            o.workspace = self.workspace.data_ptr()
            o.workspace_bytes = self.workspace.numel() * self.workspace.element_size()
        o.boundary = self.boundary
        o.hdiff_form = self.hdiff_form
        o.tile_order = self.tile_order
        if self.coeff_field is not None:
            cf = self.coeff_field if isinstance(self.coeff_field, _lib.StencilField) else self.coeff_field.c()
            o._coeff_field = cf  # keep the descriptor alive with the options
            o.coeff_field = ctypes.pointer(cf)
        return o


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return F64
    if t == torch.float32:
        return F32
    raise StencilError(-2, f"unsupported dtype {t}")


def _fld(f):
    if f is None:
        return None
    if isinstance(f, _lib.StencilField):
        return ctypes.byref(f)
    return ctypes.byref(f.c())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _opts(o):
    if o is None:
        return None
    if isinstance(o, _lib.StencilOptions):
        return ctypes.byref(o)
    return ctypes.byref(o.c())


def _stream(s) -> Optional[int]:
    if s is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _dt(dtype, *fields) -> int:
    if dtype is not None:
        return dtype if isinstance(dtype, int) else _dtype_code(dtype)
    for f in fields:
        if isinstance(f, Field):
            return _dtype_code(f.dtype)
    raise StencilError(-2, "cannot infer the dtype")


# ------------------------------------------------------------------ info
def stencil_version() -> int:
    return _lib.lib().stencil_version()


def stencil_last_error() -> str:
    return _lib.last_error()


def stencil_max_fused_nk(dtype=F64) -> int:
    return _lib.lib().stencil_max_fused_nk(_dt(dtype))


def stencil_mask_bytes(domain) -> int:
    return _lib.lib().stencil_mask_bytes(_lib.domain3(domain))


def stencil_workspace_bytes(op: int, dtype, domain, opts=None) -> int:
    return _lib.lib().stencil_workspace_bytes(op, _dt(dtype), _lib.domain3(domain), _opts(opts))


# ------------------------------------------------------------------ forward
def stencil_hdiff(u, out, domain, coeff, mask=None, opts=None, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_hdiff(_dt(dtype, u, out), _fld(u), _fld(out), _lib.domain3(domain),
                                        float(coeff), _ptr(mask), _opts(opts), _stream(stream)))


def stencil_vadv(u, data, w, out, domain, dt_dz, opts=None, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_vadv(_dt(dtype, u, out), _fld(u), _fld(data), _fld(w), _fld(out),
                                       _lib.domain3(domain), float(dt_dz), _opts(opts), _stream(stream)))


def stencil_step(u, data, w, out, domain, coeff, dt_dz, mask=None, opts=None, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_step(_dt(dtype, u, out), _fld(u), _fld(data), _fld(w), _fld(out),
                                       _lib.domain3(domain), float(coeff), float(dt_dz), _ptr(mask),
                                       _opts(opts), _stream(stream)))


# ------------------------------------------------------------------ adjoint
def stencil_hdiff_adjoint(out_bar, mask, u_bar, domain, coeff, opts=None, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_hdiff_adjoint(_dt(dtype, out_bar, u_bar), _fld(out_bar), _ptr(mask),
                                                _fld(u_bar), _lib.domain3(domain), float(coeff),
                                                _opts(opts), _stream(stream)))


def stencil_vadv_adjoint(x_bar, w, d_bar, domain, dt_dz, opts=None, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_vadv_adjoint(_dt(dtype, x_bar, d_bar), _fld(x_bar), _fld(w), _fld(d_bar),
                                               _lib.domain3(domain), float(dt_dz), _opts(opts),
                                               _stream(stream)))


def stencil_step_adjoint(x_bar, w, mask, u_bar, data_bar, domain, coeff, dt_dz, opts=None, stream=None,
                         dtype=None):
    _lib.check(_lib.lib().stencil_step_adjoint(_dt(dtype, x_bar, u_bar), _fld(x_bar), _fld(w), _ptr(mask),
                                               _fld(u_bar), _fld(data_bar), _lib.domain3(domain),
                                               float(coeff), float(dt_dz), _opts(opts), _stream(stream)))


def stencil_halo_update(f, domain, boundary=BOUNDARY_PERIODIC, stream=None, dtype=None):
    _lib.check(_lib.lib().stencil_halo_update(_dt(dtype, f), _fld(f), _lib.domain3(domain), int(boundary),
                                              _stream(stream)))


# ------------------------------------------------------------------ parameter gradients
def stencil_param_workspace_bytes(dtype, domain) -> int:
    return _lib.lib().stencil_param_workspace_bytes(_dt(dtype), _lib.domain3(domain))


def stencil_step_param_adjoint(u, w, x, lam, w_bar, coeff_bar, domain, dt_dz, ws=None, stream=None,
                               dtype=None, opts=None):
    """coeff_bar: a device tensor holding one float64 (or None); w_bar: a
    staggered field (or None); ws: the workspace tensor for coeff_bar."""
    nb = 0 if ws is None else ws.numel() * ws.element_size()
    _lib.check(_lib.lib().stencil_step_param_adjoint(
        _dt(dtype, lam), _fld(u), _fld(w), _fld(x), _fld(lam), _fld(w_bar), _ptr(coeff_bar),
        _lib.domain3(domain), float(dt_dz), _opts(opts), _ptr(ws), nb, _stream(stream)))


def stencil_coeff_field_adjoint(u, lam, kappa_bar, domain, opts=None, stream=None, dtype=None):
    """kappa_bar(p) = -lam(p) D(u)(p): the gradient of a per-point coefficient."""
    _lib.check(_lib.lib().stencil_coeff_field_adjoint(
        _dt(dtype, lam, kappa_bar), _fld(u), _fld(lam), _fld(kappa_bar), _lib.domain3(domain), _opts(opts),
        _stream(stream)))


# ------------------------------------------------------------------ batched
def _batch_items(items):
    arr = (_lib.StencilBatchItem * len(items))()
    for n, it in enumerate(items):
        arr[n].u = it["u"].c()
        arr[n].data = it["data"].c()
        arr[n].w = it["w"].c()
        arr[n].out = it["out"].c()
        arr[n].domain = _lib.domain3(it["domain"])
        arr[n].coeff = float(it["coeff"])
        arr[n].dt_dz = float(it["dt_dz"])
        arr[n].mask = _ptr(it.get("mask"))
    return arr


def _batch_adj_items(items):
    arr = (_lib.StencilBatchAdjointItem * len(items))()
    for n, it in enumerate(items):
        arr[n].x_bar = it["x_bar"].c()
        arr[n].w = it["w"].c()
        arr[n].u_bar = it["u_bar"].c()
        if it.get("data_bar") is not None:
            arr[n].data_bar = it["data_bar"].c()
        arr[n].domain = _lib.domain3(it["domain"])
        arr[n].coeff = float(it["coeff"])
        arr[n].dt_dz = float(it["dt_dz"])
        arr[n].mask = _ptr(it.get("mask"))
    return arr


def stencil_batch_workspace_bytes(dtype, items) -> int:
    arr = _batch_items(items)
    return _lib.lib().stencil_batch_workspace_bytes(_dt(dtype), len(items), arr)


def stencil_batch_adjoint_workspace_bytes(dtype, items) -> int:
    arr = _batch_adj_items(items)
    return _lib.lib().stencil_batch_adjoint_workspace_bytes(_dt(dtype), len(items), arr)


def stencil_step_batched(dtype, items, ws, opts=None, stream=None):
    arr = _batch_items(items)
    nb = 0 if ws is None else ws.numel() * ws.element_size()
    _lib.check(_lib.lib().stencil_step_batched(_dt(dtype), len(items), arr, _ptr(ws), nb, _opts(opts),
                                               _stream(stream)))


def stencil_step_batched_noalloc(dtype, items, opts=None, stream=None):
    arr = _batch_items(items)
    _lib.check(_lib.lib().stencil_step_batched_noalloc(_dt(dtype), len(items), arr, _opts(opts),
                                                       _stream(stream)))


def stencil_step_adjoint_batched(dtype, items, ws, opts=None, stream=None):
    arr = _batch_adj_items(items)
    nb = 0 if ws is None else ws.numel() * ws.element_size()
    _lib.check(_lib.lib().stencil_step_adjoint_batched(_dt(dtype), len(items), arr, _ptr(ws), nb,
                                                       _opts(opts), _stream(stream)))


# ------------------------------------------------------------------ graph
def stencil_graph_capture_steps(nsteps, u_a, u_b, data, w, domain, coeff, dt_dz, opts=None, stream=None,
                                dtype=None) -> int:
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().stencil_graph_capture_steps(
        _dt(dtype, u_a, u_b), int(nsteps), _fld(u_a), _fld(u_b), _fld(data), _fld(w), _lib.domain3(domain),
        float(coeff), float(dt_dz), _opts(opts), _stream(stream), ctypes.byref(h)))
    return h.value


def stencil_graph_launch(graph: int, stream=None):
    _lib.check(_lib.lib().stencil_graph_launch(graph, _stream(stream)))


def stencil_graph_destroy(graph: int):
    _lib.check(_lib.lib().stencil_graph_destroy(graph))


# ------------------------------------------------------------------ tuning
def stencil_autotune(dtype, op, domain, reps=5) -> float:
    us = ctypes.c_double()
    _lib.check(_lib.lib().stencil_autotune(_dt(dtype), int(op), _lib.domain3(domain), int(reps),
                                           ctypes.byref(us)))
    return us.value


def stencil_autotune_fields(u, data, w, out, domain, reps=5, op=OP_STEP, stream=None, dtype=None) -> float:
    """Tune the step on these fields (out is overwritten); returns the best time in us."""
    us = ctypes.c_double()
    _lib.check(_lib.lib().stencil_autotune_fields(_dt(dtype, u, out), int(op), _fld(u), _fld(data), _fld(w),
                                                  _fld(out), _lib.domain3(domain), int(reps), _stream(stream),
                                                  ctypes.byref(us)))
    return us.value


def stencil_tuning_lookup(dtype, op, domain):
    """(tile_i, tile_j, column_store, tile_order) chosen for this size class."""
    ti, tj, col, order = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.lib().stencil_tuning_lookup(_dt(dtype), int(op), _lib.domain3(domain), ctypes.byref(ti),
                                                ctypes.byref(tj), ctypes.byref(col), ctypes.byref(order)))
    return ti.value, tj.value, col.value, order.value


def stencil_save_tuning(path: str):
    _lib.check(_lib.lib().stencil_save_tuning(path.encode()))


def stencil_load_tuning(path: str):
    _lib.check(_lib.lib().stencil_load_tuning(path.encode()))


def stencil_clear_tuning():
    _lib.check(_lib.lib().stencil_clear_tuning())
