"""The closed form of tests/lattice_pattern.py against the oracle on sizes it
bins in milliseconds: fewer particles than bins, exact multiples, ragged
tails, several attributes."""
import numpy as np
import pytest

from oracle import binning_oracle as orc
from tests import lattice_pattern as L


@pytest.mark.parametrize("n,nx,ny,k", [(0, 8, 4, 1), (5, 8, 4, 2), (32, 8, 4, 3), (97, 8, 4, 4), (1000, 16, 16, 1),
                                       (3 * 64 + 2, 64, 1, 2), (70_001, 64, 32, 3)])
def test_closed_form_equals_oracle(n, nx, ny, k):
    idx = np.arange(n, dtype=np.int64)
    x, y, attrs = L.columns(idx, nx, ny, k, lambda v: v.astype(np.float32))
    ref = orc.bin_particles([x, y], attrs, (0, 1), (0.0, 1.0, 0.0, 1.0), nx, ny)
    exp = L.expected(n, nx, ny, k)
    assert np.array_equal(ref["count"], exp["count"])
    for key in ("sum", "min", "max", "avg", "abs_sum"):
        for j in range(k):
            assert np.array_equal(ref[key][j], exp[key][j], equal_nan=True), (key, j)


@pytest.mark.parametrize("n,nx,ny,k,f64", [(0, 8, 4, 1, False), (1, 8, 4, 1, False), (7, 8, 4, 2, False),
                                           (32, 8, 4, 1, False), (50, 37, 5, 3, True), (1000, 64, 64, 1, False),
                                           (999, 1_000_003, 1, 2, True)])
def test_sparse_closed_form_equals_oracle(n, nx, ny, k, f64):
    idx = np.arange(n, dtype=np.int64)
    cast = (lambda v: v.astype(np.float64)) if f64 else (lambda v: v.astype(np.float32))
    x, y, attrs = L.sparse_columns(idx, n, nx, ny, k, cast)
    attrs = [a.astype(np.float32) for a in attrs]
    ref = orc.bin_particles([x, y], attrs, (0, 1), (0.0, 1.0, 0.0, 1.0), nx, ny)
    exp = L.sparse_expected(n, nx, ny, k)
    assert np.array_equal(ref["count"], exp["count"])
    for key in ("sum", "min", "max", "avg", "abs_sum"):
        for j in range(k):
            assert np.array_equal(ref[key][j], exp[key][j], equal_nan=True), (key, j)


@pytest.mark.parametrize("n,nx,ny,f64", L.MAX_GRID_CASES, ids=L.MAX_GRID_IDS)
def test_sparse_pattern_bins_on_largest_grids(n, nx, ny, f64):
    """On the largest grids the oracle cannot allocate here, its index rule
    still puts every particle of the sparse pattern inside, in its cell."""
    idx = np.arange(n, dtype=np.int64)
    cast = (lambda v: v.astype(np.float64)) if f64 else (lambda v: v.astype(np.float32))
    x, y, _ = L.sparse_columns(idx, n, nx, ny, 0, cast)
    inside, bins = orc.flat_bins([x, y], (0, 1), (0.0, 1.0, 0.0, 1.0), nx, ny)
    assert inside.all()
    assert np.array_equal(bins, L.sparse_cells(idx, n, nx, ny))
    assert np.all(np.diff(bins) > 0)  # one particle per used cell
    assert bins[-1] >= nx * ny - nx  # the last row is used


@pytest.mark.parametrize("n,nx,ny,nz,k", [(0, 4, 2, 8, 1), (37, 4, 2, 8, 2), (64, 4, 2, 8, 1), (5000, 8, 16, 4, 3)])
def test_three_axis_closed_form_equals_oracle(n, nx, ny, nz, k):
    idx = np.arange(n, dtype=np.int64)
    x, y, z, attrs = L.columns3(idx, nx, ny, nz, k, lambda v: v.astype(np.float32))
    ref = orc.bin_particles_nd([x, y, z], attrs, (0, 1, 2), (0.0, 1.0) * 3, (nx, ny, nz))
    exp = L.expected3(n, nx, ny, nz, k)
    assert np.array_equal(ref["count"], exp["count"])
    for key in ("sum", "min", "max", "avg", "abs_sum"):
        for j in range(k):
            assert np.array_equal(ref[key][j], exp[key][j], equal_nan=True), (key, j)


@pytest.mark.parametrize("n,nx,ny,k", [(32, 8, 4, 1), (97, 8, 4, 4), (1000, 16, 16, 1), (3 * 64 + 2, 64, 1, 2),
                                       (70_001, 64, 32, 3), (5000, 2048, 2, 1)])
def test_closed_form_with_bounds_from_the_data(n, nx, ny, k):
    """With n >= nx * ny every cell centre occurs, the bounds from the data
    run from the first centre to the last, and each particle keeps its cell
    (the last centre sits on the closed upper edge): the closed form holds."""
    idx = np.arange(n, dtype=np.int64)
    x, y, attrs = L.columns(idx, nx, ny, k, lambda v: v.astype(np.float32))
    ref = orc.bin_particles([x, y], attrs, (0, 1), None, nx, ny)
    exp = L.expected(n, nx, ny, k)
    assert np.array_equal(ref["count"], exp["count"])
    for key in ("sum", "min", "max", "avg", "abs_sum"):
        for j in range(k):
            assert np.array_equal(ref[key][j], exp[key][j], equal_nan=True), (key, j)
