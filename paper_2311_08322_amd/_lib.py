"""ctypes view of ``libgt4mi.so`` (the C ABI declared in ``include/stencil.h``).

Argument marshalling only.  The library is looked up next to this file and
loaded on first use; if it is missing every entry point raises -- there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgt4mi.so")

F32, F64 = 0, 1

OK = 0
ERRORS = {
    -1: "STENCIL_E_NULL",
    -2: "STENCIL_E_DTYPE",
    -3: "STENCIL_E_SHAPE",
    -4: "STENCIL_E_HALO",
    -5: "STENCIL_E_STRIDE",
    -6: "STENCIL_E_ALIAS",
    -7: "STENCIL_E_WORKSPACE",
    -8: "STENCIL_E_UNSUPPORTED",
    -9: "STENCIL_E_HIP",
    -10: "STENCIL_E_ARG",
}
CODES = {v: k for k, v in ERRORS.items()}

# size of the library's fixed work-list array (stencil_step_batched_noalloc)
NOALLOC_SCRATCH_BYTES = 65536

IMPL_AUTO, IMPL_FUSED, IMPL_PLAIN = 0, 1, 2
COLUMN_AUTO, COLUMN_REGISTERS, COLUMN_OUTBUF, COLUMN_SPLIT = 0, 1, 2, 3
BOUNDARY_FROZEN, BOUNDARY_PERIODIC = 0, 1
HDIFF_STATED, HDIFF_DAMPING = 0, 1
ORDER_AUTO, ORDER_XCD, ORDER_DISPATCH = 0, 1, 2
OP_HDIFF, OP_VADV, OP_STEP, OP_HDIFF_ADJOINT, OP_VADV_ADJOINT, OP_STEP_ADJOINT = range(6)

I64x3 = ctypes.c_int64 * 3


class StencilField(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("shape", I64x3), ("stride", I64x3), ("origin", I64x3)]


class StencilOptions(ctypes.Structure):
    _fields_ = [
        ("impl", ctypes.c_int32),
        ("tile_i", ctypes.c_int32),
        ("tile_j", ctypes.c_int32),
        ("column_store", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("boundary", ctypes.c_int32),
        ("hdiff_form", ctypes.c_int32),
        ("coeff_field", ctypes.POINTER(StencilField)),
        ("tile_order", ctypes.c_int32),
    ]


class StencilBatchItem(ctypes.Structure):
    _fields_ = [
        ("u", StencilField),
        ("data", StencilField),
        ("w", StencilField),
        ("out", StencilField),
        ("domain", I64x3),
        ("coeff", ctypes.c_double),
        ("dt_dz", ctypes.c_double),
        ("mask", ctypes.c_void_p),
    ]


class StencilBatchAdjointItem(ctypes.Structure):
    _fields_ = [
        ("x_bar", StencilField),
        ("w", StencilField),
        ("u_bar", StencilField),
        ("data_bar", StencilField),
        ("domain", I64x3),
        ("coeff", ctypes.c_double),
        ("dt_dz", ctypes.c_double),
        ("mask", ctypes.c_void_p),
    ]


class StencilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


# the ABI this binding marshals for (stencil_version() of the library)
ABI_VERSION = 3

_lock = threading.Lock()
_lib = None

PF = ctypes.POINTER(StencilField)
PO = ctypes.POINTER(StencilOptions)
PI64 = ctypes.POINTER(ctypes.c_int64)
PI32 = ctypes.POINTER(ctypes.c_int32)
VP = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
SZ = ctypes.c_size_t

SIGNATURES = {
    "stencil_version": (I, []),
    "stencil_last_error": (ctypes.c_char_p, []),
    "stencil_max_fused_nk": (I, [I]),
    "stencil_mask_bytes": (SZ, [PI64]),
    "stencil_workspace_bytes": (SZ, [I, I, PI64, PO]),
    "stencil_hdiff": (I, [I, PF, PF, PI64, D, VP, PO, VP]),
    "stencil_vadv": (I, [I, PF, PF, PF, PF, PI64, D, PO, VP]),
    "stencil_step": (I, [I, PF, PF, PF, PF, PI64, D, D, VP, PO, VP]),
    "stencil_hdiff_adjoint": (I, [I, PF, VP, PF, PI64, D, PO, VP]),
    "stencil_vadv_adjoint": (I, [I, PF, PF, PF, PI64, D, PO, VP]),
    "stencil_step_adjoint": (I, [I, PF, PF, VP, PF, PF, PI64, D, D, PO, VP]),
    "stencil_param_workspace_bytes": (SZ, [I, PI64]),
    "stencil_halo_update": (I, [I, PF, PI64, I, VP]),
    "stencil_step_param_adjoint": (I, [I, PF, PF, PF, PF, PF, VP, PI64, D, PO, VP, SZ, VP]),
    "stencil_coeff_field_adjoint": (I, [I, PF, PF, PF, PI64, PO, VP]),
    "stencil_batch_workspace_bytes": (SZ, [I, I, ctypes.POINTER(StencilBatchItem)]),
    "stencil_batch_adjoint_workspace_bytes": (SZ, [I, I, ctypes.POINTER(StencilBatchAdjointItem)]),
    "stencil_step_batched": (I, [I, I, ctypes.POINTER(StencilBatchItem), VP, SZ, PO, VP]),
    "stencil_step_adjoint_batched": (I, [I, I, ctypes.POINTER(StencilBatchAdjointItem), VP, SZ, PO, VP]),
    "stencil_step_batched_noalloc": (I, [I, I, ctypes.POINTER(StencilBatchItem), PO, VP]),
    "stencil_graph_capture_steps": (I, [I, I, PF, PF, PF, PF, PI64, D, D, PO, VP, ctypes.POINTER(VP)]),
    "stencil_graph_launch": (I, [VP, VP]),
    "stencil_graph_destroy": (I, [VP]),
    "stencil_autotune": (I, [I, I, PI64, I, ctypes.POINTER(D)]),
    "stencil_autotune_fields": (I, [I, I, PF, PF, PF, PF, PI64, I, VP, ctypes.POINTER(D)]),
    "stencil_tuning_lookup": (I, [I, I, PI64, PI32, PI32, PI32, PI32]),
    "stencil_save_tuning": (I, [ctypes.c_char_p]),
    "stencil_load_tuning": (I, [ctypes.c_char_p]),
    "stencil_clear_tuning": (I, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(
                        f"{LIB_PATH} is missing: build the HIP library first "
                        "(python -m paper_2311_08322_amd.build_lib); there is no CPU fallback")
                L = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(L, name)
                    fn.restype = res
                    fn.argtypes = args
                if L.stencil_version() != ABI_VERSION:
                    raise RuntimeError(f"{LIB_PATH} has ABI {L.stencil_version()}, this binding needs "
                                       f"{ABI_VERSION}: rebuild the library")
                _lib = L
    return _lib


def last_error() -> str:
    return lib().stencil_last_error().decode(errors="replace")


def check(rc: int) -> None:
    if rc != OK:
        raise StencilError(rc, last_error())


def domain3(domain) -> I64x3:
    d = I64x3(*[int(x) for x in domain])
    return d
