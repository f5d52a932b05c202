"""Shared test helpers: device fields from oracle-layout arrays, error norms,
and the unpacking of the library's documented mask layout."""
from __future__ import annotations

import numpy as np
import torch

from paper_2311_08322_amd import fields

TOL = {torch.float64: 1e-12, torch.float32: 2e-5}


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """||got - ref||_inf / ||ref||_inf (0 if both are empty or zero)."""
    if ref.size == 0:
        return 0.0
    den = np.max(np.abs(ref))
    num = np.max(np.abs(np.asarray(got, np.float64) - ref))
    if den == 0.0:
        return float(num)
    return float(num / den)


def round_f32(a: np.ndarray) -> np.ndarray:
    return a.astype(np.float32).astype(np.float64)


def c_scalar(x: float, dtype) -> float:
    """The scalar as the kernel sees it (binary32 kernels round it once)."""
    return float(np.float32(x)) if dtype == torch.float32 else float(x)


def _r256(b: int) -> int:
    return (b + 255) // 256 * 256


def unpack_mask(mask: torch.Tensor, ni: int, nj: int, nk: int):
    """Library mask -> oracle layout (mx (nk, nj, ni+1), my (nk, nj+1, ni)).

    Layout as documented in include/stencil.h: X and Y bit planes of
    uint64[nk][nj][ceil(ni/64)] (bit b of word q is i = 64 q + b), then the
    X edge uint8[nk][nj] and the Y edge uint8[nk][ni], sections 256-B aligned.
    """
    b = mask.cpu().numpy().view(np.uint8)
    W = (ni + 63) // 64
    plane = _r256(8 * W * nj * nk)
    ex_off = 2 * plane
    ey_off = ex_off + _r256(nj * nk)

    def bits(off):
        words = b[off:off + 8 * W * nj * nk].view(np.uint64).reshape(nk, nj, W)
        bb = np.unpackbits(words.view(np.uint8).reshape(nk, nj, W, 8), axis=-1, bitorder="little")
        return bb.reshape(nk, nj, W * 64)[:, :, :ni]

    mx = np.zeros((nk, nj, ni + 1), np.uint8)
    my = np.zeros((nk, nj + 1, ni), np.uint8)
    mx[:, :, 1:] = bits(0)
    mx[:, :, 0] = b[ex_off:ex_off + nj * nk].reshape(nk, nj)
    my[:, 1:, :] = bits(plane)
    my[:, 0, :] = b[ey_off:ey_off + ni * nk].reshape(nk, ni)
    return mx, my


def dev_fields(f, dtype, device="cuda", aligned=True):
    """u (padded), data, w as device fields of `dtype`."""
    u = fields.from_padded(f.u, dtype, device, aligned=aligned)
    data = fields.from_interior(f.data, dtype, device, aligned=aligned)
    w = fields.from_interior(f.w, dtype, device, aligned=aligned)
    return u, data, w


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).numpy()
