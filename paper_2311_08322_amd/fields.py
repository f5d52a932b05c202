"""Storages: device fields laid out for the gfx950 kernels (GT4Py's storages,
Sec. 2.2, choose layout, alignment and padding per backend; these do the
same for this one).

Layout (k, j, i), unit stride along i.  Fields read with a halo get their
first interior point on a 128-byte boundary (origin_i = 128 B / element
size) and a row pitch that is a multiple of 128 bytes, so interior rows map
onto whole cache lines.  Only allocation and copies live here -- no stencil
arithmetic.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Field

HALO = 2
LINE = 128  # bytes


def _round(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def alloc(ni, nj, nk, dtype=torch.float64, device="cuda", halo=HALO, kextra=0, aligned=True,
          fill=None) -> Field:
    """A field of interior ni x nj x (nk + kextra) with `halo` points in i and j."""
    es = torch.empty((), dtype=dtype).element_size()
    a = LINE // es
    if halo and aligned:
        oi = _round(halo, a)
        pitch = _round(oi + ni + halo, a)
    elif aligned:
        oi = 0
        pitch = _round(max(ni, 1), a)
    else:
        oi = halo
        pitch = ni + 2 * halo
    rows = nj + 2 * halo
    shape = (nk + kextra, rows, pitch)
    t = torch.empty(shape, dtype=dtype, device=device) if fill is None else \
        torch.full(shape, fill, dtype=dtype, device=device)
    return Field(t, (oi, halo, 0))


def padded(f: Field, ni, nj, nk, halo=HALO) -> torch.Tensor:
    """View (nk, nj + 2 halo, ni + 2 halo) of the domain plus its halo."""
    oi, oj, ok = f.origin
    return f.tensor[ok:ok + nk, oj - halo:oj + nj + halo, oi - halo:oi + ni + halo]


def interior(f: Field, ni, nj, nk) -> torch.Tensor:
    oi, oj, ok = f.origin
    return f.tensor[ok:ok + nk, oj:oj + nj, oi:oi + ni]


def from_padded(a: np.ndarray, dtype=torch.float64, device="cuda", aligned=True) -> Field:
    """Copy an (nk, nj+4, ni+4) host array into a new device field."""
    nk, Nj, Ni = a.shape
    ni, nj = Ni - 2 * HALO, Nj - 2 * HALO
    f = alloc(ni, nj, nk, dtype, device, HALO, aligned=aligned, fill=0.0)
    padded(f, ni, nj, nk).copy_(torch.as_tensor(a).to(dtype))
    return f


def from_interior(a: np.ndarray, dtype=torch.float64, device="cuda", aligned=True) -> Field:
    """Copy an (nk', nj, ni) host array (interior or staggered) into a new field."""
    nk, nj, ni = a.shape
    f = alloc(ni, nj, nk, dtype, device, halo=0, aligned=aligned, fill=0.0)
    interior(f, ni, nj, nk).copy_(torch.as_tensor(a).to(dtype))
    return f


def mask_tensor(domain, device="cuda") -> torch.Tensor:
    from .api import stencil_mask_bytes

    return torch.zeros(max(stencil_mask_bytes(domain), 1), dtype=torch.uint8, device=device)


def workspace(op, dtype, domain, opts=None, device="cuda"):
    from .api import stencil_workspace_bytes

    n = stencil_workspace_bytes(op, dtype, domain, opts)
    return torch.empty(n, dtype=torch.uint8, device=device) if n else None
