"""GPU parity of the stencils written in the frontend's language (the
benchmark stencils of Sec. 3.1, compiled by the generated-HIP backend)
against the oracle: hdiff (stated and damping forms), vadv, the time step,
at ragged sizes, unaligned layouts and the full 512 x 512 x 80 step; domain
deduction; a refused call surfaces as an error.  In FP64 the generated
arithmetic is operation-for-operation the oracle's (no contraction), so the
values agree to the last bit."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import fields, inputs
from paper_2311_08322_amd.frontend import StencilRunError
from paper_2311_08322_amd.frontend import stencils as S

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = [torch.float64, torch.float32]
IDS = ["f64", "f32"]


def _r(a, dtype):
    return round_f32(a) if dtype == torch.float32 else a


def _check(got, want, dtype):
    assert rel_err(got, want) <= TOL[dtype]
    if dtype == torch.float64:
        assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("damping", [False, True], ids=["stated", "damping"])
@pytest.mark.parametrize("aligned", [True, False], ids=["aligned", "packed"])
@pytest.mark.parametrize("dims", [(67, 45, 7), (1, 1, 3), (130, 5, 4), (256, 256, 8)],
                         ids=lambda d: "x".join(map(str, d)))
def test_hdiff(dims, aligned, damping, dtype):
    ni, nj, nk = dims
    print(f"frontend hdiff {dims} aligned={aligned} damping={damping} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=700)
    u = fields.from_padded(f.u, dtype, DEV, aligned=aligned)
    out = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, aligned=aligned, fill=0.0)
    st = S.hdiff_damping if damping else S.hdiff
    st(u, out, coeff=inputs.COEFF, domain=dims)
    torch.cuda.synchronize()
    want, _, _ = orc.hdiff(_r(f.u, dtype), c_scalar(inputs.COEFF, dtype), decide_f32=(dtype == torch.float32),
                           damping=damping)
    _check(host(fields.interior(out, ni, nj, nk)), want[:, 2:-2, 2:-2], dtype)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("dims", [(64, 64, 16), (67, 45, 7), (5, 3, 1), (9, 7, 2), (33, 17, 137), (20, 20, 200)],
                         ids=lambda d: "x".join(map(str, d)))
def test_vadv(dims, dtype):
    ni, nj, nk = dims
    print(f"frontend vadv {dims} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=701)
    uin = inputs.cotangent(ni, nj, nk, child=702)
    u = fields.from_interior(uin, dtype, DEV)
    data = fields.from_interior(f.data, dtype, DEV)
    w = fields.from_interior(f.w, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    S.vadv(u, data, w, out, dt_dz=inputs.DT_DZ, domain=dims)
    torch.cuda.synchronize()
    want = orc.vadv(_r(uin, dtype), _r(f.data, dtype), _r(f.w, dtype), inputs.DT_DZ)
    _check(host(fields.interior(out, ni, nj, nk)), want, dtype)


@pytest.mark.parametrize("dtype", DTYPES, ids=IDS)
@pytest.mark.parametrize("dims", [(64, 64, 16), (67, 45, 7), (1, 1, 1), (130, 3, 97), (33, 17, 170)],
                         ids=lambda d: "x".join(map(str, d)))
def test_step(dims, dtype):
    ni, nj, nk = dims
    print(f"frontend step {dims} {dtype}", flush=True)
    f = inputs.fields_sized(ni, nj, nk, seed=703)
    u, data, w = dev_fields(f, dtype, DEV)
    out = fields.alloc(ni, nj, nk, dtype, DEV, halo=0, fill=0.0)
    S.step(u, data, w, out, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, domain=dims)
    torch.cuda.synchronize()
    nxt, _, _ = orc.step(_r(f.u, dtype), _r(f.data, dtype), _r(f.w, dtype), c_scalar(inputs.COEFF, dtype),
                         inputs.DT_DZ, decide_f32=(dtype == torch.float32))
    _check(host(fields.interior(out, ni, nj, nk)), nxt[:, 2:-2, 2:-2], dtype)


def test_step_full_size_and_domain_deduction():
    """512 x 512 x 80 FP64 with the domain deduced from the fields (u's
    halo, w's extra level), bit for bit the oracle's step."""
    dims = (512, 512, 80)
    ni, nj, nk = dims
    f = inputs.fields_for(inputs.STEP_512)
    u, data, w = dev_fields(f, torch.float64, DEV)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    got_dom = S.step(u, data, w, out, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ)
    torch.cuda.synchronize()
    assert got_dom == dims
    nxt, _, _ = orc.step(f.u, f.data, f.w, inputs.COEFF, inputs.DT_DZ)
    assert np.array_equal(host(fields.interior(out, ni, nj, nk)), nxt[:, 2:-2, 2:-2])


def test_refused_call_raises():
    """A u without the 2-point halo the stencil reads is refused by the
    generated library before any launch."""
    ni, nj, nk = 16, 12, 4
    u = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=1, fill=0.0)
    out = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    with pytest.raises(StencilRunError):
        S.hdiff(u, out, coeff=0.025, domain=(ni, nj, nk))


def test_step_on_two_streams():
    """The generated step on two side streams at once (each call with its own
    workspace) equals the default-stream result bit for bit."""
    ni, nj, nk = 96, 64, 40
    dims = (ni, nj, nk)
    f = inputs.fields_sized(ni, nj, nk, seed=704)
    u, data, w = dev_fields(f, torch.float64, DEV)
    ref = fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0)
    S.step(u, data, w, ref, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, domain=dims)
    outs = [fields.alloc(ni, nj, nk, torch.float64, DEV, halo=0, fill=0.0) for _ in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    torch.cuda.synchronize()
    for o, s in zip(outs, streams):
        for _ in range(3):
            S.step(u, data, w, o, coeff=inputs.COEFF, dt_dz=inputs.DT_DZ, domain=dims, stream=s)
    torch.cuda.synchronize()
    want = host(fields.interior(ref, ni, nj, nk))
    for o in outs:
        assert np.array_equal(host(fields.interior(o, ni, nj, nk)), want)
