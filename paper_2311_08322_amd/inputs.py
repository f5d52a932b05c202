"""Seeded synthetic inputs for the stencil workloads.

This module only draws random numbers and names sizes: it holds none of the
stencils' arithmetic, so both the HIP path (through the tests and the
benchmark) and the CPU reference can take their inputs from it.

Recipe (the paper publishes no fields or domain sizes; the workloads are the
two benchmark stencils of Sec. 3.1 at the sizes below):

* one ``numpy.random.SeedSequence(20231108)``; workload ``n`` draws from
  child ``n``; cotangents from child 100, dot-test vectors from child 101,
  finite-difference probe points from child 102;
* arrays are drawn in FP64 in the order u, w, data:
  ``u ~ U[0,1)`` on the padded (halo 2) domain, corners included;
  ``w ~ U[-1,1]`` on nk+1 staggered levels; ``data ~ U[-0.1,0.1]``;
* binary32 runs use ``astype(float32)`` of the same draws;
* scalars: coeff = 0.025, dt/dz = 0.5;
* a per-point coefficient field (the generalised diffusion) is drawn
  ``U[coeff/2, 3 coeff/2)`` on the interior from child 103;
* the batched workload draws 32 (ni, nj, nk) triples, integers uniform and
  inclusive in [48,384] x [48,384] x [40,137], then one child per field;
* domains too large for host arrays (levels beyond 2 GiB) are drawn on the
  device by torch's generator, seeded from child 104 (fields, the same
  ranges) and 105 (cotangent), in the fields' own precision.

Arrays are returned in the layout (k, j, i) with i fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ROOT_SEED = 20231108
HALO = 2
COEFF = 0.025
DT_DZ = 0.5


@dataclass(frozen=True)
class Workload:
    name: str
    ni: int
    nj: int
    nk: int
    child: int  # SeedSequence child index


# The five benchmark workloads (sizes of the interior; halo 2 in i and j).
HDIFF_64 = Workload("hdiff 64x64x16", 64, 64, 16, 1)
STEP_256 = Workload("hdiff+vadv 256x256x80", 256, 256, 80, 2)
STEP_512 = Workload("fused step 512x512x80", 512, 512, 80, 3)
ADJ_256 = Workload("step adjoint 256x256x80", 256, 256, 80, 4)
BATCH_CHILD = 5
BATCH_FIELDS = 32
BATCH_RANGE = ((48, 384), (48, 384), (40, 137))

LARGE_CHILD = 104  # fields drawn on the device (domains too large for host arrays)

COTANGENT_CHILD = 100
DOT_CHILD = 101
FD_CHILD = 102
COEFF_FIELD_CHILD = 103


def _children(n: int):
    return np.random.SeedSequence(ROOT_SEED).spawn(n + 1)


def rng_for(child: int) -> np.random.Generator:
    """Generator for SeedSequence child `child` of the root seed."""
    return np.random.default_rng(_children(child)[child])


@dataclass
class Fields:
    u: np.ndarray  # (nk, nj+4, ni+4)
    w: np.ndarray  # (nk+1, nj, ni)
    data: np.ndarray  # (nk, nj, ni)

    @property
    def dims(self):
        nk, nj, ni = self.data.shape
        return ni, nj, nk


def draw_fields(ni: int, nj: int, nk: int, rng: np.random.Generator) -> Fields:
    u = rng.random((nk, nj + 2 * HALO, ni + 2 * HALO))
    w = rng.uniform(-1.0, 1.0, (nk + 1, nj, ni))
    data = rng.uniform(-0.1, 0.1, (nk, nj, ni))
    return Fields(u=u, w=w, data=data)


def fields_for(wl: Workload) -> Fields:
    return draw_fields(wl.ni, wl.nj, wl.nk, rng_for(wl.child))


def fields_sized(ni: int, nj: int, nk: int, seed: int) -> Fields:
    """Same distributions at an arbitrary size, from child `seed`."""
    return draw_fields(ni, nj, nk, rng_for(seed))


def cotangent(ni: int, nj: int, nk: int, child: int = COTANGENT_CHILD) -> np.ndarray:
    return rng_for(child).uniform(-1.0, 1.0, (nk, nj, ni))


def dot_vectors(ni: int, nj: int, nk: int):
    """v on the padded domain, w on the interior, both U[-1,1]."""
    r = rng_for(DOT_CHILD)
    v = r.uniform(-1.0, 1.0, (nk, nj + 2 * HALO, ni + 2 * HALO))
    wv = r.uniform(-1.0, 1.0, (nk, nj, ni))
    return v, wv


def coeff_field(ni: int, nj: int, nk: int, child: int = COEFF_FIELD_CHILD) -> np.ndarray:
    """Per-point diffusion coefficient on the interior, U[coeff/2, 3 coeff/2)."""
    return rng_for(child).uniform(0.5 * COEFF, 1.5 * COEFF, (nk, nj, ni))


def fd_points(ni: int, nj: int, nk: int, count: int = 64) -> np.ndarray:
    """`count` distinct flat indices into the padded (nk, nj+4, ni+4) array."""
    n = nk * (nj + 2 * HALO) * (ni + 2 * HALO)
    return rng_for(FD_CHILD).choice(n, size=min(count, n), replace=False)


def batch_sizes(n: int = BATCH_FIELDS):
    r = rng_for(BATCH_CHILD)
    (i0, i1), (j0, j1), (k0, k1) = BATCH_RANGE
    out = []
    for _ in range(n):
        ni = int(r.integers(i0, i1, endpoint=True))
        nj = int(r.integers(j0, j1, endpoint=True))
        nk = int(r.integers(k0, k1, endpoint=True))
        out.append((ni, nj, nk))
    return out


def batch_fields(n: int = BATCH_FIELDS):
    """List of (ni, nj, nk, Fields) for the batched uneven workload."""
    sizes = batch_sizes(n)
    seeds = np.random.SeedSequence([ROOT_SEED, BATCH_CHILD]).spawn(len(sizes))
    res = []
    for (ni, nj, nk), s in zip(sizes, seeds):
        res.append((ni, nj, nk, draw_fields(ni, nj, nk, np.random.default_rng(s))))
    return res


def as_f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _torch_seed(child: int) -> int:
    return int(np.random.SeedSequence([ROOT_SEED, child]).generate_state(1, np.uint64)[0] >> 1)


def fill_device(views, ranges, child: int) -> None:
    """Fills device tensors (views allowed) in order, view n uniform on
    ranges[n] = (lo, hi), from torch's generator on their device seeded from
    the child's SeedSequence: for domains whose arrays are too large to draw
    on the host.  The values are drawn in the views' own precision; a CPU
    check reads back the values actually stored, so both sides see the same
    inputs."""
    import torch

    g = torch.Generator(device=views[0].device)
    g.manual_seed(_torch_seed(child))
    for v, (lo, hi) in zip(views, ranges):
        v.uniform_(lo, hi, generator=g)


# the ranges of u, w and data (as draw_fields) and of a cotangent
FIELD_RANGES = ((0.0, 1.0), (-1.0, 1.0), (-0.1, 0.1))
COTANGENT_RANGE = (-1.0, 1.0)
