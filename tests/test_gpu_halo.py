"""Periodic boundaries on the GPU: the halo update equals the oracle's fill
bit for bit, a periodic step equals the oracle's step followed by the fill,
the graph loop with periodic boundaries equals eager steps and is consistent
with the oracle step by step, and periodic diffusion conserves the interior
sum."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = [torch.float64, torch.float32]
IDS = ["f64", "f32"]
PERIODIC = api.Options(boundary=api.BOUNDARY_PERIODIC)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("aligned", [True, False], ids=["aligned", "packed"])
@pytest.mark.parametrize("dims", [(67, 45, 7), (1, 1, 3), (2, 3, 2), (130, 5, 4), (256, 256, 8)],
                         ids=lambda d: "x".join(map(str, d)))
def test_halo_update_matches_oracle(dims, aligned, dtype):
    ni, nj, nk = dims
    print(f"halo update {dims} aligned={aligned} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=500)
    u = fields.from_padded(f.u, dtype, DEV, aligned=aligned)
    api.stencil_halo_update(u, dims)
    torch.cuda.synchronize()
    src = round_f32(f.u) if dtype == torch.float32 else f.u
    assert np.array_equal(host(fields.padded(u, ni, nj, nk)), orc.halo_periodic(src))


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
def test_periodic_step(dtype):
    ni, nj, nk = 97, 43, 17
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=501)
    up = orc.halo_periodic(f.u)
    u = fields.from_padded(up, dtype, DEV)
    data = fields.from_interior(f.data, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, fill=-5.0)
    api.stencil_step(u, data, w, out, dims, inputs.COEFF, inputs.DT_DZ, opts=PERIODIC)
    torch.cuda.synchronize()
    r = round_f32 if dtype == torch.float32 else (lambda a: a)
    nxt, _, _ = orc.step(r(up), r(f.data), r(f.w), c_scalar(inputs.COEFF, dtype), inputs.DT_DZ,
                         decide_f32=(dtype == torch.float32))
    got = host(fields.padded(out, ni, nj, nk))
    assert rel_err(got[:, 2:-2, 2:-2], nxt[:, 2:-2, 2:-2]) <= TOL[dtype]
    # the halo is the periodic fill of the GPU's own new interior
    assert np.array_equal(got, orc.halo_periodic(got))


def test_periodic_graph_matches_eager_and_oracle():
    """A 10-step periodic graph equals 10 eager periodic steps bit for bit;
    each eager step n is consistent with the oracle applied to state n-1
    (then filled), and every state's halo is the fill of its interior."""
    dtype = torch.float64
    ni, nj, nk = 128, 96, 24
    dims = (ni, nj, nk)
    nsteps = 10
    f = inputs.fields_sized(ni, nj, nk, seed=502)
    up = orc.halo_periodic(f.u)
    data = fields.from_interior(f.data, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    u_a = fields.from_padded(up, dtype, DEV)
    u_b = fields.from_padded(up, dtype, DEV)
    e = [fields.from_padded(up, dtype, DEV), fields.from_padded(up, dtype, DEV)]
    states = [up]
    for n in range(nsteps):
        src, dst = e[n % 2], e[(n + 1) % 2]
        api.stencil_step(src, data, w, dst, dims, inputs.COEFF, inputs.DT_DZ, opts=PERIODIC)
        torch.cuda.synchronize()
        states.append(host(fields.padded(dst, ni, nj, nk)))
    for n in range(1, nsteps + 1):
        prev, cur = states[n - 1], states[n]
        assert np.array_equal(cur, orc.halo_periodic(cur)), n
        nxt, _, _ = orc.step(prev, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
        assert rel_err(cur[:, 2:-2, 2:-2], nxt[:, 2:-2, 2:-2]) <= TOL[dtype], n
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = api.stencil_graph_capture_steps(nsteps, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ,
                                            opts=PERIODIC, stream=s)
    try:
        api.stencil_graph_launch(g, stream=s)
        s.synchronize()
        res = u_b if nsteps % 2 else u_a
        assert np.array_equal(host(fields.padded(res, ni, nj, nk)), states[-1])
    finally:
        api.stencil_graph_destroy(g)


def test_periodic_diffusion_conserves_mass():
    """w = 0 and data = 0: the column solve is the identity and periodic
    diffusion telescopes, so 50 graph steps keep the interior sum."""
    dtype = torch.float64
    ni, nj, nk = 256, 192, 8
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=503)
    up = orc.halo_periodic(f.u)
    u_a = fields.from_padded(up, dtype, DEV)
    u_b = fields.from_padded(up, dtype, DEV)
    data = fields.from_interior(np.zeros_like(f.data), dtype, DEV)
    w = fields.from_interior(np.zeros_like(f.w), dtype, DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = api.stencil_graph_capture_steps(50, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ,
                                            opts=PERIODIC, stream=s)
    try:
        api.stencil_graph_launch(g, stream=s)
        s.synchronize()
    finally:
        api.stencil_graph_destroy(g)
    x = host(fields.interior(u_a, ni, nj, nk))  # 50 steps: the state is back in u_a
    s0 = math.fsum(up[:, 2:-2, 2:-2].ravel())
    s1 = math.fsum(x.ravel())
    assert abs(s1 - s0) <= 1e-12 * math.fsum(np.abs(x).ravel())
    assert not np.array_equal(x, up[:, 2:-2, 2:-2])  # it did diffuse
