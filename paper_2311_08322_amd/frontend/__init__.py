"""A GTScript-like stencil frontend for the gfx950 backend.

Write a stencil as a Python function (GT4Py paper, Sec. 2.2)::

    from paper_2311_08322_amd.frontend import (Field, stencil, function, computation,
                                               interval, PARALLEL, FORWARD, BACKWARD)

    @function
    def lap(f):
        return 4.0 * f - (f[-1, 0, 0] + f[1, 0, 0] + f[0, -1, 0] + f[0, 1, 0])

    @stencil
    def smooth(u: Field, out: Field, *, alpha: float):
        with computation(PARALLEL), interval(...):
            out = u - alpha * lap(u)

``smooth(u, out, alpha=0.1)`` takes ``api.Field`` objects (a torch tensor
laid out (k, j, i) plus the origin of the domain in it), deduces the domain
from the field sizes and the stencil's extents unless ``domain=`` is given,
and runs the generated HIP library (built once per definition and dtype,
cached under a fingerprint; ``.build(dtype)`` builds ahead of time).  There
is no interpreter fallback: every call runs the compiled kernels.
"""
from __future__ import annotations

import ctypes
import inspect
from typing import Dict, Optional

import torch

from . import build as _build
from . import ir
from .analysis import StencilAnalysisError, analyse
from .hipgen import CodegenError
from .parse import GTScriptSyntaxError, function_ast, parse_stencil

PARALLEL, FORWARD, BACKWARD = ir.PARALLEL, ir.FORWARD, ir.BACKWARD

__all__ = ["Field", "stencil", "function", "computation", "interval", "PARALLEL", "FORWARD", "BACKWARD",
           "StencilObject", "GTScriptSyntaxError", "StencilAnalysisError", "CodegenError", "StencilRunError"]


class _FieldAnnotation:
    """Marker for field parameters (``u: Field`` or ``u: Field[float]``)."""

    def __getitem__(self, item):
        return self


Field = _FieldAnnotation()


def computation(order):  # pragma: no cover - only parsed, never executed
    raise RuntimeError("computation() is GTScript syntax: call the decorated stencil instead")


def interval(*args):  # pragma: no cover
    raise RuntimeError("interval() is GTScript syntax: call the decorated stencil instead")


class StencilRunError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stencil run failed ({code}): {msg}")
        self.code = code


class Function:
    """A ``@function``: inlined where a stencil (or another function) calls it."""

    def __init__(self, fn):
        self.fn = fn
        self.name = fn.__name__
        self.ast = function_ast(fn)

    def __call__(self, *a, **k):  # pragma: no cover
        raise RuntimeError("a @function is inlined into stencils, not called from Python")


def function(fn):
    return Function(fn)


def _functions_visible(fn) -> Dict[str, Function]:
    out = {}
    scope = dict(fn.__globals__)
    cv = inspect.getclosurevars(fn)
    scope.update(cv.nonlocals)
    for k, v in scope.items():
        if isinstance(v, Function):
            out[k] = v
    return out


class StencilObject:
    def __init__(self, fn, externals=None):
        self.fn = fn
        self.externals = dict(externals or {})
        self.definition = parse_stencil(fn, self.externals, _functions_visible(fn))
        self.plan = analyse(self.definition)
        self._libs = {}

    @property
    def name(self):
        return self.definition.name

    def fingerprint(self, dtype="float64"):
        return _build.fingerprint(self.definition, dtype)

    def source(self, dtype="float64"):
        from . import hipgen
        return hipgen.generate(self.plan, dtype, self.fingerprint(dtype))

    def build(self, dtype="float64", force=False):
        key = dtype
        if key not in self._libs or force:
            self._libs[key] = _build.load(_build.compile_library(self.definition, dtype, force))
        return self._libs[key]

    # ------------------------------------------------------------ calling
    def extents(self):
        """Per API field: (ilo, ihi, jlo, jhi) offsets it is read at."""
        return {n: f.ext for n, f in self.plan.fields.items()}

    def __call__(self, *args, domain=None, origin=None, stream=None, **scalars):
        sd = self.definition
        if len(args) != len(sd.fields):
            raise TypeError(f"{sd.name} takes {len(sd.fields)} fields, got {len(args)}")
        for s in sd.scalars:
            if s not in scalars:
                raise TypeError(f"{sd.name}: missing scalar {s}")
        extra = set(scalars) - set(sd.scalars)
        if extra:
            raise TypeError(f"{sd.name}: unknown arguments {sorted(extra)}")
        fl = []
        dtype = None
        for name, a in zip(sd.fields, args):
            t = a.tensor if hasattr(a, "tensor") else a
            o = tuple(a.origin) if hasattr(a, "origin") else (0, 0, 0)
            if isinstance(origin, dict) and name in origin:
                o = tuple(origin[name])
            elif origin is not None and not isinstance(origin, dict):
                o = tuple(origin)
            if not isinstance(t, torch.Tensor) or t.dim() != 3:
                raise TypeError(f"field {name}: a 3-D tensor laid out (k, j, i)")
            if dtype is None:
                dtype = t.dtype
            elif t.dtype != dtype:
                raise TypeError(f"field {name}: dtype {t.dtype} differs from {dtype}")
            fl.append((name, t, o))
        dts = {torch.float64: "float64", torch.float32: "float32"}.get(dtype)
        if dts is None:
            raise TypeError(f"dtype {dtype} unsupported")
        if domain is None:
            d = [None, None, None]
            for name, t, o in fl:
                e = self.plan.fields[name].ext if self.plan.fields[name].read else (0, 0, 0, 0)
                shp = (t.shape[2], t.shape[1], t.shape[0])
                cand = (shp[0] - o[0] - e[1], shp[1] - o[1] - e[3], shp[2] - o[2])
                d = [c if x is None else min(x, c) for x, c in zip(d, cand)]
            domain = tuple(max(0, x) for x in d)
        domain = tuple(int(x) for x in domain)
        L = self.build(dts)
        arr = (_build.GtsField * max(1, len(fl)))()
        for idx, (name, t, o) in enumerate(fl):
            shp = (t.shape[2], t.shape[1], t.shape[0])
            st = (t.stride(2), t.stride(1), t.stride(0))
            f = arr[idx]
            f.data = t.data_ptr() + (o[0] * st[0] + o[1] * st[1] + o[2] * st[2]) * t.element_size()
            for ax in range(3):
                f.stride[ax] = st[ax]
                f.lo[ax] = o[ax]
                f.hi[ax] = shp[ax] - o[ax]
        sc = (ctypes.c_double * max(1, len(sd.scalars)))(*[float(scalars[s]) for s in sd.scalars])
        dom = (ctypes.c_int64 * 3)(*domain)
        nb = L.gts_workspace_bytes(dom)
        if stream is None:
            ts = torch.cuda.current_stream() if torch.cuda.is_available() else None
        elif isinstance(stream, int):
            ts = torch.cuda.ExternalStream(stream)
        else:
            ts = stream
        s = ts.cuda_stream if ts is not None else None
        ws = None
        if nb:
            # one workspace per call from torch's caching allocator, tied to the
            # stream the kernels run on (overlapping calls never share one)
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=fl[0][1].device)
            if ts is not None and ts != torch.cuda.current_stream():
                ws.record_stream(ts)
        wp = 0 if ws is None else (ws.data_ptr() + 255) // 256 * 256
        rc = L.gts_run(arr, len(fl), sc, len(sd.scalars), dom, wp or None, nb, s)
        if rc != 0:
            raise StencilRunError(rc, L.gts_last_error().decode(errors="replace"))
        return domain


def stencil(fn=None, *, externals: Optional[dict] = None):
    """Decorator: ``@stencil`` or ``@stencil(externals={...})``."""
    if fn is None:
        return lambda f: StencilObject(f, externals)
    return StencilObject(fn, externals)
