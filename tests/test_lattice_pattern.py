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
