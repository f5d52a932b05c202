"""GPU check of stencil_step_batched_noalloc, the batched forward step whose
work list lives in the library's fixed device array instead of a caller
workspace.  Two calls in a row, the second on a smaller batch (so the array
still holds the first call's longer table), each compared bit for bit with
stencil_step_batched on the same inputs (the same kernels and tiles), masks
included, and the smaller batch also against the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2311_08322_amd import api, fields, inputs

from .helpers import TOL, c_scalar, dev_fields, host, rel_err, round_f32, unpack_mask

pytestmark = pytest.mark.gpu
DEV = "cuda"

# first call: uneven fields, FP64 columns on both sides of the 80-level
# split of the batched kernels, ragged tile edges; second call: fewer and
# smaller fields
FIRST = [(96, 80, 88), (130, 70, 40), (48, 48, 137), (200, 64, 81), (64, 96, 120), (50, 61, 60)]
SECOND = [(40, 33, 20), (20, 9, 30)]


def _items(sizes, seed, dtype, masks):
    items, host_fields = [], []
    for n, (ni, nj, nk) in enumerate(sizes):
        f = inputs.fields_sized(ni, nj, nk, seed=seed + n)
        u, data, w = dev_fields(f, dtype, DEV)
        dims = (ni, nj, nk)
        items.append(dict(u=u, data=data, w=w, out=fields.alloc(ni, nj, nk, dtype, DEV, fill=0.0), domain=dims,
                          coeff=inputs.COEFF, dt_dz=inputs.DT_DZ,
                          mask=fields.mask_tensor(dims, DEV) if masks[n % len(masks)] else None))
        host_fields.append(f)
    return items, host_fields


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_batch_matches_workspace_batch(dtype):
    for call, (sizes, seed) in enumerate(((FIRST, 7100), (SECOND, 7200))):
        print(f"no-alloc batch, call {call}, {dtype}, sizes {sizes}", flush=True)
        masks = (True, False)
        a, hf = _items(sizes, seed, dtype, masks)
        b, _ = _items(sizes, seed, dtype, masks)
        assert api.stencil_batch_workspace_bytes(dtype, a) <= api._lib.NOALLOC_SCRATCH_BYTES
        api.stencil_step_batched_noalloc(dtype, a)
        ws = torch.empty(api.stencil_batch_workspace_bytes(dtype, b), dtype=torch.uint8, device=DEV)
        api.stencil_step_batched(dtype, b, ws)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            ni, nj, nk = x["domain"]
            assert torch.equal(fields.interior(x["out"], ni, nj, nk), fields.interior(y["out"], ni, nj, nk)), \
                (call, x["domain"])
            if x["mask"] is not None:
                assert torch.equal(x["mask"], y["mask"]), (call, x["domain"])
        if call == 1:  # the smaller batch against the oracle too
            f32 = dtype == torch.float32
            for x, f in zip(a, hf):
                ni, nj, nk = x["domain"]
                r = inputs.Fields(u=round_f32(f.u), w=round_f32(f.w), data=round_f32(f.data)) if f32 else f
                nxt, mx, my = orc.step(r.u, r.data, r.w, c_scalar(inputs.COEFF, dtype), inputs.DT_DZ,
                                       decide_f32=f32)
                err = rel_err(host(fields.interior(x["out"], ni, nj, nk)), nxt[:, 2:-2, 2:-2])
                assert err <= TOL[dtype], (x["domain"], err)
                if x["mask"] is not None:
                    gx, gy = unpack_mask(x["mask"], ni, nj, nk)
                    assert np.array_equal(gx, mx) and np.array_equal(gy, my), x["domain"]
