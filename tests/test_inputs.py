"""The seeded generators are deterministic and follow the stated recipe."""
import numpy as np

from paper_2311_08322_amd import inputs


def test_deterministic_and_shaped():
    a = inputs.fields_sized(9, 7, 5, seed=3)
    b = inputs.fields_sized(9, 7, 5, seed=3)
    c = inputs.fields_sized(9, 7, 5, seed=4)
    assert a.u.shape == (5, 11, 13) and a.w.shape == (6, 7, 9) and a.data.shape == (5, 7, 9)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.w, b.w) and np.array_equal(a.data, b.data)
    assert not np.array_equal(a.u, c.u)
    assert a.dims == (9, 7, 5)


def test_distributions():
    f = inputs.fields_sized(64, 64, 16, seed=1)
    assert 0.0 <= f.u.min() and f.u.max() < 1.0
    assert -1.0 <= f.w.min() and f.w.max() <= 1.0 and f.w.min() < -0.9 and f.w.max() > 0.9
    assert -0.1 <= f.data.min() and f.data.max() <= 0.1
    assert abs(f.u.mean() - 0.5) < 0.01


def test_workloads():
    assert (inputs.STEP_512.ni, inputs.STEP_512.nj, inputs.STEP_512.nk) == (512, 512, 80)
    assert (inputs.HDIFF_64.ni, inputs.HDIFF_64.nk) == (64, 16)
    f = inputs.fields_for(inputs.HDIFF_64)
    g = inputs.fields_for(inputs.HDIFF_64)
    assert np.array_equal(f.u, g.u)


def test_batch_sizes_in_range():
    sizes = inputs.batch_sizes()
    assert len(sizes) == 32
    for ni, nj, nk in sizes:
        assert 48 <= ni <= 384 and 48 <= nj <= 384 and 40 <= nk <= 137
    assert sizes == inputs.batch_sizes()
    assert len(set(sizes)) > 20


def test_f32_is_rounded_f64_draw():
    f = inputs.fields_sized(8, 8, 4, seed=2)
    u32 = inputs.as_f32(f.u)
    assert u32.dtype == np.float32
    assert np.max(np.abs(u32.astype(np.float64) - f.u)) <= np.finfo(np.float32).eps


def test_fd_points_distinct():
    p = inputs.fd_points(10, 9, 4, 64)
    assert len(set(p.tolist())) == 64
    assert p.max() < 4 * 13 * 14
