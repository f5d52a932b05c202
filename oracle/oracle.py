"""NumPy front-end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; it calls only ``liboracle.so`` built from
``oracle.c`` next to this file.

Array conventions (C order, float64):
  padded  ``u``/``out``/``ubar``: (nk, nj+4, ni+4) -- halo 2 in i and j
  interior ``data``/``x``/``lam``/``xbar``: (nk, nj, ni)
  staggered ``w``: (nk+1, nj, ni)
  masks (uint8, 1 = flux kept): ``mx`` (nk, nj, ni+1) for x-fluxes with
  i in [-1, ni); ``my`` (nk, nj+1, ni) for y-fluxes with j in [-1, nj).

``decide_f32`` makes the limiter decision in binary32 (values stay FP64), so
that the oracle branches exactly as a binary32 kernel does on the same
binary32 inputs.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP: independent levels / columns over the
# host's threads, identical arithmetic (CPU baseline on all cores)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC"]


def _build_one(path: str, extra) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, *extra, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, path)


def build(force: bool = True) -> str:
    """Compile liboracle.so (and its OpenMP twin) with gcc: plain loops, no
    FP contraction."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            _build_one(path, extra)
    return _LIB


_libs = {}
_threaded = False


@contextlib.contextmanager
def threaded():
    """Oracle calls inside the block run on the OpenMP build (all threads
    OMP_NUM_THREADS allows); results are identical to the serial build."""
    global _threaded
    prev, _threaded = _threaded, True
    try:
        yield lib()
    finally:
        _threaded = prev


def threads() -> int:
    """Threads a parallel region of the current build uses."""
    return int(lib().oracle_threads())


def lib():
    path = _LIB_OMP if _threaded else _LIB
    if path not in _libs:
        # (re)build when missing or older than its source, so a stale
        # library never answers for the current definitions
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _build_one(path, ["-fopenmp"] if path == _LIB_OMP else [])
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        bp = ctypes.POINTER(ctypes.c_ubyte)
        I, D = ctypes.c_int, ctypes.c_double
        sig = {
            "oracle_hdiff_masks": [I, I, I, dp, I, bp, bp],
            "oracle_hdiff": [I, I, I, dp, D, I, dp, bp, bp],
            "oracle_vadv": [I, I, I, dp, dp, dp, D, dp],
            "oracle_step": [I, I, I, dp, dp, dp, D, D, I, dp, bp, bp],
            "oracle_hdiff_adjoint": [I, I, I, dp, bp, bp, D, dp],
            "oracle_vadv_adjoint": [I, I, I, dp, dp, D, dp],
            "oracle_step_adjoint": [I, I, I, dp, dp, bp, bp, D, D, dp, dp],
            "oracle_step_tangent": [I, I, I, dp, dp, bp, bp, D, D, dp],
            "oracle_hdiff_tangent": [I, I, I, dp, bp, bp, D, dp],
            "oracle_tridiag_apply": [I, I, I, dp, dp, D, dp],
            "oracle_laplacian": [I, I, I, dp, dp],
            "oracle_hdiff_divergence": [I, I, I, dp, bp, bp, dp],
            "oracle_w_grad": [I, I, I, dp, dp, dp, D, dp],
            "oracle_halo_periodic": [I, I, I, dp],
            "oracle_hdiff_masks_form": [I, I, I, dp, I, I, bp, bp],
            "oracle_hdiff_gen": [I, I, I, dp, D, dp, I, I, dp, bp, bp],
            "oracle_step_gen": [I, I, I, dp, dp, dp, D, dp, I, D, I, dp, bp, bp],
            "oracle_hdiff_adjoint_gen": [I, I, I, dp, bp, bp, D, dp, I, dp],
            "oracle_step_adjoint_gen": [I, I, I, dp, dp, bp, bp, D, dp, I, D, dp, dp],
            "oracle_step_tangent_gen": [I, I, I, dp, dp, bp, bp, D, dp, I, D, dp],
            "oracle_hdiff_tangent_gen": [I, I, I, dp, bp, bp, D, dp, I, dp],
            "oracle_hdiff_divergence_form": [I, I, I, dp, bp, bp, I, dp],
            "oracle_coeff_field_grad": [I, I, I, dp, dp, bp, bp, I, dp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        L.oracle_coeff_grad.argtypes = [I, I, I, dp, dp, bp, bp]
        L.oracle_coeff_grad.restype = D
        L.oracle_coeff_grad_form.argtypes = [I, I, I, dp, dp, bp, bp, I]
        L.oracle_coeff_grad_form.restype = D
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = I
        _libs[path] = L
    return _libs[path]


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _b(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _u8(a, shape):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _kappa(kappa, nk, nj, ni):
    """(array kept alive, pointer): the per-point coefficient field or NULL."""
    if kappa is None:
        return None, ctypes.POINTER(ctypes.c_double)()
    k = _f64(kappa, (nk, nj, ni))
    return k, _d(k)


def _dims_padded(u):
    nk, Nj, Ni = u.shape
    return Ni - 4, Nj - 4, nk


def hdiff_masks(u, decide_f32=False, damping=False):
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    mx = np.zeros((nk, nj, ni + 1), np.uint8)
    my = np.zeros((nk, nj + 1, ni), np.uint8)
    lib().oracle_hdiff_masks_form(ni, nj, nk, _d(u), int(decide_f32), int(damping), _b(mx), _b(my))
    return mx, my


def hdiff(u, coeff, decide_f32=False, kappa=None, damping=False):
    """Returns (out padded with u's halo, mx, my).  ``kappa`` (interior
    shape) replaces the scalar coeff by a per-point coefficient; ``damping``
    takes the discrete Laplacian instead of its negative."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    keep, kp = _kappa(kappa, nk, nj, ni)
    out = np.empty_like(u)
    mx = np.zeros((nk, nj, ni + 1), np.uint8)
    my = np.zeros((nk, nj + 1, ni), np.uint8)
    lib().oracle_hdiff_gen(ni, nj, nk, _d(u), float(coeff), kp, int(damping), int(decide_f32), _d(out),
                           _b(mx), _b(my))
    return out, mx, my


def vadv(uin, data, w, dt_dz):
    """x = T(w)^{-1} (uin + data); all interior arrays, w staggered."""
    nk, nj, ni = np.shape(uin)
    uin = _f64(uin, (nk, nj, ni))
    data = _f64(data, (nk, nj, ni))
    w = _f64(w, (nk + 1, nj, ni))
    x = np.zeros((nk, nj, ni))
    lib().oracle_vadv(ni, nj, nk, _d(uin), _d(data), _d(w), float(dt_dz), _d(x))
    return x


def step(u, data, w, coeff, dt_dz, decide_f32=False, kappa=None, damping=False):
    """Returns (next padded state, mx, my)."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    data = _f64(data, (nk, nj, ni))
    w = _f64(w, (nk + 1, nj, ni))
    keep, kp = _kappa(kappa, nk, nj, ni)
    nxt = np.empty_like(u)
    mx = np.zeros((nk, nj, ni + 1), np.uint8)
    my = np.zeros((nk, nj + 1, ni), np.uint8)
    lib().oracle_step_gen(ni, nj, nk, _d(u), _d(data), _d(w), float(coeff), kp, int(damping),
                          float(dt_dz), int(decide_f32), _d(nxt), _b(mx), _b(my))
    return nxt, mx, my


def hdiff_adjoint(lam, mx, my, coeff, kappa=None, damping=False):
    nk, nj, ni = np.shape(lam)
    lam = _f64(lam, (nk, nj, ni))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    keep, kp = _kappa(kappa, nk, nj, ni)
    ubar = np.zeros((nk, nj + 4, ni + 4))
    lib().oracle_hdiff_adjoint_gen(ni, nj, nk, _d(lam), _b(mx), _b(my), float(coeff), kp, int(damping),
                                   _d(ubar))
    return ubar


def vadv_adjoint(xbar, w, dt_dz):
    nk, nj, ni = np.shape(xbar)
    xbar = _f64(xbar, (nk, nj, ni))
    w = _f64(w, (nk + 1, nj, ni))
    lam = np.zeros((nk, nj, ni))
    lib().oracle_vadv_adjoint(ni, nj, nk, _d(xbar), _d(w), float(dt_dz), _d(lam))
    return lam


def step_adjoint(xbar, w, mx, my, coeff, dt_dz, kappa=None, damping=False):
    """Returns (ubar padded, databar interior)."""
    nk, nj, ni = np.shape(xbar)
    xbar = _f64(xbar, (nk, nj, ni))
    w = _f64(w, (nk + 1, nj, ni))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    keep, kp = _kappa(kappa, nk, nj, ni)
    ubar = np.zeros((nk, nj + 4, ni + 4))
    dbar = np.zeros((nk, nj, ni))
    lib().oracle_step_adjoint_gen(ni, nj, nk, _d(xbar), _d(w), _b(mx), _b(my), float(coeff), kp,
                                  int(damping), float(dt_dz), _d(ubar), _d(dbar))
    return ubar, dbar


def step_tangent(v, w, mx, my, coeff, dt_dz, kappa=None, damping=False):
    ni, nj, nk = _dims_padded(v)
    v = _f64(v, (nk, nj + 4, ni + 4))
    w = _f64(w, (nk + 1, nj, ni))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    keep, kp = _kappa(kappa, nk, nj, ni)
    dx = np.zeros((nk, nj, ni))
    lib().oracle_step_tangent_gen(ni, nj, nk, _d(v), _d(w), _b(mx), _b(my), float(coeff), kp,
                                  int(damping), float(dt_dz), _d(dx))
    return dx


def hdiff_tangent(v, mx, my, coeff, kappa=None, damping=False):
    ni, nj, nk = _dims_padded(v)
    v = _f64(v, (nk, nj + 4, ni + 4))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    keep, kp = _kappa(kappa, nk, nj, ni)
    dh = np.zeros((nk, nj, ni))
    lib().oracle_hdiff_tangent_gen(ni, nj, nk, _d(v), _b(mx), _b(my), float(coeff), kp, int(damping),
                                   _d(dh))
    return dh


def tridiag_apply(x, w, dt_dz):
    nk, nj, ni = np.shape(x)
    x = _f64(x, (nk, nj, ni))
    w = _f64(w, (nk + 1, nj, ni))
    y = np.zeros((nk, nj, ni))
    lib().oracle_tridiag_apply(ni, nj, nk, _d(x), _d(w), float(dt_dz), _d(y))
    return y


def laplacian(u):
    """The Laplacian stage on the box [-1, ni] x [-1, nj]: (nk, nj+2, ni+2)."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    lap = np.zeros((nk, nj + 2, ni + 2))
    lib().oracle_laplacian(ni, nj, nk, _d(u), _d(lap))
    return lap


def hdiff_divergence(u, mx, my, damping=False):
    """D(u): the divergence of the limited fluxes on the interior."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    div = np.zeros((nk, nj, ni))
    lib().oracle_hdiff_divergence_form(ni, nj, nk, _d(u), _b(mx), _b(my), int(damping), _d(div))
    return div


def coeff_grad(u, lam, mx, my, damping=False):
    """dL/dcoeff = -sum lam * D(u) (compensated sum)."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    lam = _f64(lam, (nk, nj, ni))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    return float(lib().oracle_coeff_grad_form(ni, nj, nk, _d(u), _d(lam), _b(mx), _b(my), int(damping)))


def coeff_field_grad(u, lam, mx, my, damping=False):
    """dL/dkappa(p) = -lam(p) D(u)(p) for a per-point coefficient field."""
    ni, nj, nk = _dims_padded(u)
    u = _f64(u, (nk, nj + 4, ni + 4))
    lam = _f64(lam, (nk, nj, ni))
    mx = _u8(mx, (nk, nj, ni + 1))
    my = _u8(my, (nk, nj + 1, ni))
    kbar = np.zeros((nk, nj, ni))
    lib().oracle_coeff_field_grad(ni, nj, nk, _d(u), _d(lam), _b(mx), _b(my), int(damping), _d(kbar))
    return kbar


def w_grad(w, x, lam, dt_dz):
    """dL/dw on the nk+1 staggered levels (x: the step output, interior)."""
    nk, nj, ni = np.shape(x)
    w = _f64(w, (nk + 1, nj, ni))
    x = _f64(x, (nk, nj, ni))
    lam = _f64(lam, (nk, nj, ni))
    wbar = np.zeros((nk + 1, nj, ni))
    lib().oracle_w_grad(ni, nj, nk, _d(w), _d(x), _d(lam), float(dt_dz), _d(wbar))
    return wbar


def halo_periodic(u):
    """A copy of the padded array u with its 2-point halo filled periodically
    from the interior (corners included)."""
    ni, nj, nk = _dims_padded(u)
    v = _f64(u, (nk, nj + 4, ni + 4)).copy()
    lib().oracle_halo_periodic(ni, nj, nk, _d(v))
    return v
