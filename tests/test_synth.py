"""Seeded generators: determinism and the structure each workload promises."""
import numpy as np

from oracle import binning_oracle as orc
from paper_2310_02926_amd import synth


def test_uniform_f64_deterministic():
    a = synth.uniform_f64(4096, seed=0)
    b = synth.uniform_f64(4096, seed=0)
    c = synth.uniform_f64(4096, seed=1)
    assert all(np.array_equal(p, q) for p, q in zip(a.coords + a.attrs, b.coords + b.attrs))
    assert not np.array_equal(a.coords[0], c.coords[0])
    assert a.coords[0].dtype == np.float64 and a.attrs[0].dtype == np.float64
    assert np.all(a.attrs[0] > 0)


def test_gmm_outside_share_exact():
    w = synth.gmm_f32(n=200_000, seed=0, nx=64, ny=64, k=4)
    x, y = w.coords
    assert x.dtype == np.float32 and len(w.attrs) == 4
    inside = (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)
    assert int((~inside).sum()) == round(0.02 * 200_000) == w.meta["n_outside"]
    r = orc.bin_particles(w.coords, w.attrs[:1], (0, 1), (0, 1, 0, 1), 64, 64)
    assert r["inside"] == int(inside.sum())
    # clustered: the busiest 10% of bins hold well over 10% of the particles
    c = np.sort(r["count"].ravel())[::-1]
    assert c[: c.size // 10].sum() > 0.3 * c.sum()
    w2 = synth.gmm_f32(n=200_000, seed=0, nx=64, ny=64, k=4)
    assert np.array_equal(w.coords[1], w2.coords[1]) and np.array_equal(w.attrs[3], w2.attrs[3])


def test_hotspot_share():
    side = 256
    w = synth.hotspot_f32(n=400_000, seed=0, side=side)
    r = orc.bin_particles(w.coords, w.attrs, (0, 1), (0, 1, 0, 1), side, side)
    hot = w.meta["hot_bins"]
    assert hot.size == int(0.01 * side * side)
    c = r["count"].ravel()
    assert c[hot].sum() >= 0.9 * 400_000
    assert r["inside"] == 400_000
    # hot particles sit strictly inside their bin (margin 0.05 of a cell)
    assert np.all(w.attrs[0] > 0)


def test_batch_specs_ranges():
    specs = synth.batch_specs(256, seed=0)
    assert len(specs) == 256
    assert all(1000 <= s.n <= 10_000_000 for s in specs)
    assert all(s.side in synth.BATCH_SIDES for s in specs)
    assert all(1 <= s.k <= 4 and 0 < s.ops < 32 for s in specs)
    assert specs[0].n == synth.batch_specs(256, seed=0)[0].n


def test_poisson_arrivals():
    t = synth.poisson_arrivals(1000.0, 20000, seed=0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 1e-3) < 5e-5


def test_halos3d_shape_and_determinism():
    a = synth.halos3d_f32(100_000, seed=3, side=16)
    b = synth.halos3d_f32(100_000, seed=3, side=16)
    assert all(np.array_equal(x, y) for x, y in zip(a.coords, b.coords))
    assert len(a.coords) == 3 and all(c.dtype == np.float32 and c.size == 100_000 for c in a.coords)
    axes, bounds, dims = a.meta["nd"]
    assert axes == (0, 1, 2) and dims == (16, 16, 16)
    inside = np.ones(100_000, bool)
    for c in a.coords:
        inside &= (c >= 0) & (c <= 1)
    # the background reaches past the cube, so some particles are outside
    assert 0.005 < 1 - inside.mean() < 0.2
