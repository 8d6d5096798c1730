"""Seeded input generators: shapes, distinct coordinates, value sets, skew
and reproducibility."""
import numpy as np
import pytest

from paper_2003_03572_amd import gen


def _lin(idx, dims):
    i = idx.astype(np.int64)
    return (i[:, 0] * dims[1] + i[:, 1]) * dims[2] + i[:, 2]


def test_small_uniform_shape_values_and_distinct():
    dims, idx, vals = gen.make(gen.SMALL_UNIFORM)
    assert dims == (200, 150, 100)
    assert idx.shape == (20_000, 3) and idx.dtype == np.int32
    assert vals.dtype == np.float32
    assert set(np.unique(vals).tolist()) == {1.0, 2.0, 3.0, 4.0, 5.0}
    for n in range(3):
        assert idx[:, n].min() >= 0 and idx[:, n].max() < dims[n]
    assert np.unique(_lin(idx, dims)).size == 20_000


def test_reproducible_and_seed_dependent():
    a = gen.make(gen.SMALL_UNIFORM)
    b = gen.make(gen.SMALL_UNIFORM)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    c = gen.uniform_distinct_linear((200, 150, 100), 20_000, 1002)
    assert not np.array_equal(a[1], c[1])


def test_zipf_head_mass_matches_pmf():
    rng = np.random.Generator(np.random.PCG64(5))
    n, length, alpha = 400_000, 1000, 1.2
    x = gen.zipf_indices(rng, n, length, alpha)
    pmf = np.arange(1, length + 1, dtype=np.float64) ** -alpha
    pmf /= pmf.sum()
    for i in range(5):
        p = pmf[i]
        assert abs((x == i).mean() - p) < 5 * np.sqrt(p * (1 - p) / n)
    assert x.min() >= 0 and x.max() < length


def test_zipf_tensor_distinct_exact_count():
    dims, idx, vals = gen.zipf_coords((1000, 500, 50), 50_000, 1.2, seed=7)
    assert idx.shape == (50_000, 3)
    assert np.unique(_lin(idx, dims)).size == 50_000
    # skew: index 0 is the most popular in every mode
    for n in range(3):
        counts = np.bincount(idx[:, n], minlength=dims[n])
        assert counts.argmax() == 0


def test_uniform_coords_exp_values():
    dims, idx, vals = gen.uniform_coords((300, 300, 50), 100_000, seed=3)
    assert np.unique(_lin(idx, dims)).size == 100_000
    assert vals.min() > 0 and abs(vals.mean() - 1.0) < 0.02


def test_job_specs_ranges():
    specs = gen.job_specs(64)
    for s in specs:
        assert all(50 <= d <= 5000 for d in s.dims)
        assert 1 <= s.nnz_target <= 1_000_000
        assert s.nnz_target <= 0.2 * s.dims[0] * s.dims[1] * s.dims[2]
        assert s.rank in (8, 16, 32, 64)


def test_scaled_workload_keeps_structure():
    dims, idx, vals = gen.make(gen.ZIPF_UIT, scale=1e-3)
    assert idx.shape[0] == 10_000
    assert all(d >= 4 for d in dims)
