"""The hipGraph-captured time loop: replay equals eager launches bitwise,
the halo stays frozen, and every step is consistent with the oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("nsteps", [1, 6, 11])
def test_graph_replay_matches_eager(nsteps, dtype):
    ni, nj, nk = 96, 40, 24
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=301)
    u_a, data, w = dev_fields(f, dtype, DEV)
    u_b = fields.from_padded(f.u, dtype, DEV)  # same halo in both buffers
    e_a = fields.from_padded(f.u, dtype, DEV)
    e_b = fields.from_padded(f.u, dtype, DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = api.stencil_graph_capture_steps(nsteps, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ,
                                            stream=s)
    try:
        # eager reference on the default stream
        for n in range(nsteps):
            src, dst = (e_a, e_b) if n % 2 == 0 else (e_b, e_a)
            api.stencil_step(src, data, w, dst, dims, inputs.COEFF, inputs.DT_DZ)
        torch.cuda.synchronize()
        eager = e_b if nsteps % 2 else e_a
        for rep in range(3):  # replays are independent of earlier eager work
            pa = fields.padded(u_a, ni, nj, nk)
            pb = fields.padded(u_b, ni, nj, nk)
            pa.copy_(torch.as_tensor(f.u, device=DEV).to(dtype))
            pb.copy_(torch.as_tensor(f.u, device=DEV).to(dtype))
            torch.cuda.synchronize()
            api.stencil_graph_launch(g, stream=s)
            s.synchronize()
            res = u_b if nsteps % 2 else u_a
            assert torch.equal(fields.padded(res, ni, nj, nk), fields.padded(eager, ni, nj, nk)), rep
        # frozen halo
        full = host(fields.padded(res, ni, nj, nk))
        ring = np.ones(full.shape, bool)
        ring[:, 2:-2, 2:-2] = False
        ref = f.u.astype(np.float32).astype(np.float64) if dtype == torch.float32 else f.u
        assert np.array_equal(full[ring], ref[ring])
    finally:
        api.stencil_graph_destroy(g)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_per_step_consistency_with_oracle(dtype):
    """Limiter branch flips make free runs of two correct implementations
    drift apart, so each GPU step is checked on a state the oracle produced:
    oracle state n -> one GPU step == oracle state n+1, at several n."""
    ni, nj, nk = 64, 48, 20
    f = inputs.fields_sized(ni, nj, nk, seed=302)
    coeff = c_scalar(inputs.COEFF, dtype)
    r32 = dtype == torch.float32
    state = round_f32(f.u) if r32 else f.u
    data = round_f32(f.data) if r32 else f.data
    wv = round_f32(f.w) if r32 else f.w
    dd = fields.from_interior(data, dtype, DEV)
    ww = fields.from_interior(wv, dtype, DEV)
    for n in range(12):
        nxt, _, _ = orc.step(state, data, wv, coeff, inputs.DT_DZ, decide_f32=r32)
        if n in (0, 1, 5, 11):
            src = fields.from_padded(state, dtype, DEV)
            dst = fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0)
            api.stencil_step(src, dd, ww, dst, (ni, nj, nk), inputs.COEFF, inputs.DT_DZ)
            assert rel_err(host(fields.interior(dst, ni, nj, nk)), nxt[:, 2:-2, 2:-2]) <= TOL[dtype], n
        state = round_f32(nxt) if r32 else nxt


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_graph_loop_full_size_per_step_gate(dtype):
    """The 100-step loop at 512x512x80 gated per step on its own states:
    a graph of n + 1 steps leaves state n in one ping-pong buffer and state
    n + 1 in the other, and the oracle applied to GPU state n must give GPU
    state n + 1 (1e-12 FP64, 2e-5 FP32 against the oracle fed the binary32
    state and inputs with binary32 limiter decisions), at n = 1, 50, 99."""
    wl = inputs.STEP_512
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    f = inputs.fields_for(wl)
    r32 = dtype == torch.float32
    data_r = round_f32(f.data) if r32 else f.data
    w_r = round_f32(f.w) if r32 else f.w
    coeff = c_scalar(inputs.COEFF, dtype)
    u_a, data, w = dev_fields(f, dtype, DEV)
    u_b = fields.from_padded(f.u, dtype, DEV)
    s = torch.cuda.Stream()
    for n in (1, 50, 99):
        print(f"per-step gate 512x512x80 {dtype}: graph of {n + 1} steps", flush=True)
        for buf in (u_a, u_b):
            fields.padded(buf, ni, nj, nk).copy_(torch.as_tensor(f.u, device=DEV).to(dtype))
        torch.cuda.synchronize()
        g = api.stencil_graph_capture_steps(n + 1, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ, stream=s)
        try:
            api.stencil_graph_launch(g, stream=s)
            s.synchronize()
        finally:
            api.stencil_graph_destroy(g)
        # step m writes u_b for even m (0-based), u_a for odd m
        last, prev = (u_b, u_a) if n % 2 == 0 else (u_a, u_b)
        state_n = host(fields.padded(prev, ni, nj, nk))
        state_n1 = host(fields.interior(last, ni, nj, nk))
        assert np.isfinite(state_n1).all()
        nxt, _, _ = orc.step(state_n, data_r, w_r, coeff, inputs.DT_DZ, decide_f32=r32)
        err = rel_err(state_n1, nxt[:, 2:-2, 2:-2])
        print(f"  step {n} -> {n + 1}: rel err {err:.3e}", flush=True)
        assert err <= TOL[dtype], (n, err)


def test_graph_capture_full_size_100_steps():
    """The 100-step loop at 512x512x80 FP64: graph replay == eager, bitwise."""
    wl = inputs.STEP_512
    ni, nj, nk = wl.ni, wl.nj, wl.nk
    dims = (ni, nj, nk)
    f = inputs.fields_for(wl)
    u_a, data, w = dev_fields(f, torch.float64, DEV)
    u_b = fields.from_padded(f.u, torch.float64, DEV)
    s = torch.cuda.Stream()
    g = api.stencil_graph_capture_steps(100, u_a, u_b, data, w, dims, inputs.COEFF, inputs.DT_DZ, stream=s)
    try:
        api.stencil_graph_launch(g, stream=s)
        s.synchronize()
        e_a = fields.from_padded(f.u, torch.float64, DEV)
        e_b = fields.from_padded(f.u, torch.float64, DEV)
        for n in range(100):
            src, dst = (e_a, e_b) if n % 2 == 0 else (e_b, e_a)
            api.stencil_step(src, data, w, dst, dims, inputs.COEFF, inputs.DT_DZ)
        torch.cuda.synchronize()
        assert torch.equal(fields.padded(u_a, ni, nj, nk), fields.padded(e_a, ni, nj, nk))
        x = fields.interior(u_a, ni, nj, nk)
        assert torch.isfinite(x).all() and float(x.abs().max()) < 100.0
    finally:
        api.stencil_graph_destroy(g)
