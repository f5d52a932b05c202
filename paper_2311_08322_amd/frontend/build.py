"""Fingerprint cache, compilation and loading of generated stencil libraries.

The fingerprint hashes the canonical text of the definition IR (so
reformatting, comments or renaming nothing observable reuse the cached
build; GT4Py paper, Sec. 2.3), the dtype, the generator version and the
compiler flags.  Each build lives in ``_gtcache/<name>_<dtype>_<fingerprint>/``
next to this package: the generated ``stencil.hip`` and ``libstencil.so``.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
import threading

from . import hipgen, ir
from .analysis import analyse

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
CACHE = os.environ.get("GT4MI_STENCIL_CACHE", os.path.join(PKG, "_gtcache"))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-variable",
         "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]



def fingerprint(sdef: ir.StencilDef, dtype: str) -> str:
    h = hashlib.sha256()
    h.update(repr(sdef).encode())
    h.update(dtype.encode())
    h.update(str(hipgen.GEN_VERSION).encode())
    h.update(" ".join(FLAGS[:-2]).encode())
    return h.hexdigest()[:16]


def build_dir(sdef: ir.StencilDef, dtype: str) -> str:
    return os.path.join(CACHE, f"{sdef.name}_{dtype}_{fingerprint(sdef, dtype)}")


def compile_library(sdef: ir.StencilDef, dtype: str, force: bool = False) -> str:
    """Generate and compile (unless cached); returns the library path."""
    d = build_dir(sdef, dtype)
    lib = os.path.join(d, "libstencil.so")
    if os.path.exists(lib) and not force:
        return lib
    plan = analyse(sdef)
    src = hipgen.generate(plan, dtype, fingerprint(sdef, dtype))
    os.makedirs(d, exist_ok=True)
    tag = "%d_%d" % (os.getpid(), threading.get_ident())
    path = os.path.join(d, f"stencil.hip.{tag}")
    with open(path, "w") as f:
        f.write(src)
    tmp = lib + ".tmp" + tag
    r = subprocess.run([HIPCC, *FLAGS, "-x", "hip", path, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for stencil {sdef.name} ({dtype}):\n{r.stderr[-4000:]}")
    # concurrent builders of one fingerprint write the same bytes; renames are atomic
    os.replace(path, os.path.join(d, "stencil.hip"))
    os.replace(tmp, lib)
    return lib


class GtsField(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("stride", ctypes.c_int64 * 3), ("lo", ctypes.c_int64 * 3),
                ("hi", ctypes.c_int64 * 3)]


def load(path: str):
    L = ctypes.CDLL(path)
    L.gts_run.restype = ctypes.c_int
    L.gts_run.argtypes = [ctypes.POINTER(GtsField), ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                          ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    L.gts_workspace_bytes.restype = ctypes.c_size_t
    L.gts_workspace_bytes.argtypes = [ctypes.POINTER(ctypes.c_int64)]
    L.gts_signature.restype = ctypes.c_char_p
    L.gts_last_error.restype = ctypes.c_char_p
    return L
