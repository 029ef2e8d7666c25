"""Pins that tie the CPU oracle to something other than itself.

Each ``pin_*`` takes an oracle module (the real one, or a copy with a planted
mistake) and raises AssertionError if the module disagrees with:

* the hand-worked fixtures in tests/golden/hand_cases.json,
* the exact rational brute force (index) and exactly rounded sums,
* SciPy's ``binned_statistic_2d`` and NumPy's ``histogram2d``,
* invariants and metamorphic relations of the binning definition.

The real oracle must pass all of them; every planted mistake must fail at
least one (tests/test_oracle_mutants.py).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

ALL = 31


def _num(v):
    if isinstance(v, str):
        return {"nan": math.nan, "inf": math.inf, "-inf": -math.inf, "-0": -0.0}[v]
    return float(v)


def _arr(nested):
    if isinstance(nested, list):
        return np.array([_arr(x) for x in nested])
    return _num(nested)


def same_bits(a, b) -> bool:
    """Equal as binary64 bit patterns, any NaN equal to any NaN."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        return False
    nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(nan | (a.view(np.int64) == b.view(np.int64))))


def golden_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)["cases"]


def pin_golden(orc):
    for case in golden_cases():
        cols = [np.array([_num(v) for v in case[c]]) for c in ("x", "y", "z") if c in case]
        attrs = [np.array([_num(v) for v in case[c]]) for c in ("a", "b") if c in case]
        r = orc.bin_particles(cols, attrs, tuple(case["axes"]), tuple(case["bounds"]),
                              case["nx"], case["ny"], ALL)
        name = case["name"]
        assert r["inside"] == case["inside"], name
        assert np.array_equal(r["count"], np.array(case["count"])), name
        for j in range(len(attrs)):
            assert np.array_equal(r["sum"][j], _arr(case["sum"][j])), (name, "sum", j)
            assert same_bits(r["min"][j], _arr(case["min"][j])), (name, "min", j)
            assert same_bits(r["max"][j], _arr(case["max"][j])), (name, "max", j)
            assert same_bits(r["avg"][j], _arr(case["avg"][j])), (name, "avg", j)


def _compare_to_bruteforce(orc, coords, attrs, axes, bounds, nx, ny, sum_rel=1e-13):
    r = orc.bin_particles(coords, attrs, axes, bounds, nx, ny, ALL)
    bf = orc_bruteforce(coords, attrs, axes, bounds, nx, ny)
    assert r["inside"] == bf["inside"]
    assert np.array_equal(r["count"], bf["count"])
    for j in range(len(attrs)):
        assert np.all(np.abs(r["sum"][j] - bf["sum"][j]) <= sum_rel * bf["abs_sum"][j]), "sum"
        assert np.allclose(r["abs_sum"][j], bf["abs_sum"][j], rtol=1e-13, atol=0)
        assert same_bits(r["min"][j], bf["min"][j]), "min"
        assert same_bits(r["max"][j], bf["max"][j]), "max"
        cnt = bf["count"]
        ok = np.where(cnt == 0, np.isnan(r["avg"][j]),
                      np.abs(r["avg"][j] - bf["avg"][j]) <= sum_rel * bf["abs_sum"][j] / np.maximum(cnt, 1))
        assert np.all(ok), "avg"


def orc_bruteforce(coords, attrs, axes, bounds, nx, ny):
    # The brute force is always the unmodified one: it is the independent side.
    from oracle import binning_oracle as real
    return real.bin_particles_bruteforce(coords, attrs, axes, bounds, nx, ny)


def pin_bruteforce_random(orc):
    """Random particles incl. outside ones and signed values, dyadic meshes
    (where the binary64 index formula is exact), against the rational brute force."""
    rng = np.random.default_rng(123)
    for (nx, ny, bounds, n) in [(8, 4, (0.0, 1.0, 0.0, 1.0), 600),
                                (16, 16, (-2.0, 2.0, -1.0, 1.0), 900),
                                (1, 1, (0.0, 1.0, 0.0, 1.0), 200),
                                (32, 2, (0.0, 0.5, 0.25, 0.75), 700)]:
        x = rng.uniform(bounds[0] - 0.1, bounds[1] + 0.1, n)
        y = rng.uniform(bounds[2] - 0.1, bounds[3] + 0.1, n)
        z = rng.uniform(-1, 1, n)
        a = rng.standard_normal(n) * 10
        m = rng.lognormal(0, 2, n)
        _compare_to_bruteforce(orc, [x, y, z], [a, m], (0, 1), bounds, nx, ny)
        _compare_to_bruteforce(orc, [x, y, z], [m], (1, 0), (bounds[2], bounds[3], bounds[0], bounds[1]), ny, nx)


def pin_bruteforce_edges(orc):
    """Every bin edge, its one-ulp neighbours, the bounds, NaN and +-Inf, on
    dyadic meshes: the binary64 formula must give the exact rational bin."""
    # lo = 0 keeps x - lo exact; hi - lo and n powers of two keep the scale exact.
    for (nx, lo, hi, dt) in [(8, 0.0, 1.0, np.float64), (64, 0.0, 1.0, np.float32),
                             (4, 0.0, 4.0, np.float64), (16, 0.0, 0.5, np.float64),
                             (1024, 0.0, 1.0, np.float32)]:
        dtn = np.dtype(dt)
        e = (lo + (hi - lo) * np.arange(nx + 1) / nx).astype(dtn)
        pts = np.concatenate([e, np.nextafter(e, dtn.type(-np.inf)), np.nextafter(e, dtn.type(np.inf)),
                              np.array([np.nan, np.inf, -np.inf], dtype=dtn)])
        n = pts.size
        ys = np.full(n, (lo + hi) / 2, dtype=dtn)
        vals = np.arange(1, n + 1, dtype=np.float64)
        _compare_to_bruteforce(orc, [pts, ys], [vals], (0, 1), (lo, hi, lo, hi), nx, 1)
        _compare_to_bruteforce(orc, [ys, pts], [vals], (0, 1), (lo, hi, lo, hi), 1, nx)


def pin_general_bounds_near_edges(orc):
    """Non-dyadic meshes: the binary64 formula may differ from the exact
    rational bin only for points within a few ulps of a bin edge."""
    rng = np.random.default_rng(7)
    for (nx, lo, hi) in [(3, 0.0, 1.0), (10, -0.3, 0.7), (7, 1.0, 1.1), (1000, -5.0, 3.0)]:
        x = rng.uniform(lo, hi, 3000)
        edges = [lo + (hi - lo) * i / nx for i in range(nx + 1)]
        x = np.concatenate([x, np.array(edges), np.nextafter(np.array(edges), np.inf),
                            np.nextafter(np.array(edges), -np.inf)])
        ins, idx = orc.axis_index(x, lo, hi, nx)
        from oracle import binning_oracle as real
        for i, v in enumerate(x):
            ex = real._exact_index(float(v), lo, hi, nx)
            assert (ex is not None) == bool(ins[i])
            if ex is None or ex == idx[i]:
                continue
            # a disagreement must be at an edge between the two candidate bins
            edge = lo + (hi - lo) * max(ex, int(idx[i])) / nx
            assert abs(ex - int(idx[i])) == 1
            assert abs(v - edge) <= 8 * np.spacing(max(abs(edge), abs(v), abs(lo), abs(hi)))


def pin_scipy(orc):
    """SciPy binned_statistic_2d (count/sum/min/max/mean) on dyadic meshes,
    where its linspace edges equal the binary64 index formula."""
    from scipy.stats import binned_statistic_2d
    rng = np.random.default_rng(5)
    n = 20000
    nx, ny = 32, 16
    x = rng.random(n)
    y = rng.random(n)
    x[:50] = 1.0           # closed upper edge
    y[50:100] = 1.0
    a = rng.standard_normal(n) + 0.5
    r = orc.bin_particles([x, y], [a], (0, 1), (0.0, 1.0, 0.0, 1.0), nx, ny, ALL)
    ex = np.linspace(0, 1, nx + 1)
    ey = np.linspace(0, 1, ny + 1)
    # SciPy's statistic arrays are [x][y]; ours are [y][x].
    cnt = binned_statistic_2d(x, y, None, "count", bins=[ex, ey]).statistic.T
    assert np.array_equal(r["count"], cnt.astype(np.int64))
    s = binned_statistic_2d(x, y, a, "sum", bins=[ex, ey]).statistic.T
    assert np.allclose(r["sum"][0], s, rtol=1e-12, atol=1e-12)
    mn = binned_statistic_2d(x, y, a, "min", bins=[ex, ey]).statistic.T
    mx = binned_statistic_2d(x, y, a, "max", bins=[ex, ey]).statistic.T
    mean = binned_statistic_2d(x, y, a, "mean", bins=[ex, ey]).statistic.T
    full = cnt > 0
    assert np.array_equal(r["min"][0][full], mn[full])
    assert np.array_equal(r["max"][0][full], mx[full])
    assert np.allclose(r["avg"][0][full], mean[full], rtol=1e-12, atol=1e-12)
    h, _, _ = np.histogram2d(x, y, bins=[ex, ey])
    assert np.array_equal(r["count"], h.T.astype(np.int64))


def pin_invariants(orc):
    rng = np.random.default_rng(11)
    n = 50000
    x = rng.uniform(-0.1, 1.1, n)
    y = rng.uniform(-0.1, 1.1, n)
    a = rng.standard_normal(n)
    m = rng.lognormal(0, 1, n)
    nx, ny = 20, 30
    r = orc.bin_particles([x, y], [a, m], (0, 1), (0.0, 1.0, 0.0, 1.0), nx, ny, ALL)
    inside = int(np.sum((x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)))
    assert r["inside"] == inside
    assert int(r["count"].sum()) == inside
    cnt = r["count"]
    full = cnt > 0
    for j in range(2):
        mn, mx, av, s = r["min"][j], r["max"][j], r["avg"][j], r["sum"][j]
        tol = 1e-12 * r["abs_sum"][j] / np.maximum(cnt, 1)
        assert np.all(mn[full] <= av[full] + tol[full])
        assert np.all(av[full] <= mx[full] + tol[full])
        assert np.all(np.abs(s - av * cnt)[full] <= 1e-12 * r["abs_sum"][j][full])
        assert np.all(np.isposinf(mn[~full])) and np.all(np.isneginf(mx[~full]))
        assert np.all(s[~full] == 0) and np.all(np.isnan(av[~full]))
        # the attribute total over inside particles is preserved
        keep = (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)
        assert math.isclose(s.sum(), math.fsum([a, m][j][keep]), rel_tol=1e-11)


def pin_metamorphic(orc):
    rng = np.random.default_rng(17)
    n = 30000
    x = rng.uniform(-0.05, 1.05, n)
    y = rng.uniform(-0.05, 1.05, n)
    a = rng.standard_normal(n)
    b = rng.lognormal(0, 1, n)
    nx, ny = 24, 10
    bnd = (0.0, 1.0, 0.0, 1.0)
    base = orc.bin_particles([x, y], [a, b], (0, 1), bnd, nx, ny, ALL)
    # permutation invariance: count/min/max bit-identical, sums to rounding
    p = rng.permutation(n)
    r = orc.bin_particles([x[p], y[p]], [a[p], b[p]], (0, 1), bnd, nx, ny, ALL)
    assert np.array_equal(r["count"], base["count"])
    for j in range(2):
        assert same_bits(r["min"][j], base["min"][j]) and same_bits(r["max"][j], base["max"][j])
        assert np.all(np.abs(r["sum"][j] - base["sum"][j]) <= 1e-12 * base["abs_sum"][j])
    # attribute order: results follow the attribute list
    r = orc.bin_particles([x, y], [b, a], (0, 1), bnd, nx, ny, ALL)
    assert same_bits(r["max"][0], base["max"][1]) and same_bits(r["min"][1], base["min"][0])
    # merge law over a split
    cut = n // 3
    p1 = orc.bin_particles([x[:cut], y[:cut]], [a[:cut], b[:cut]], (0, 1), bnd, nx, ny, ALL)
    p2 = orc.bin_particles([x[cut:], y[cut:]], [a[cut:], b[cut:]], (0, 1), bnd, nx, ny, ALL)
    mg = orc.merge([p1, p2])
    assert np.array_equal(mg["count"], base["count"])
    for j in range(2):
        assert same_bits(mg["min"][j], base["min"][j]) and same_bits(mg["max"][j], base["max"][j])
        assert np.all(np.abs(mg["sum"][j] - base["sum"][j]) <= 1e-12 * base["abs_sum"][j])
    # swapping the axes (and the bounds and sides with them) transposes the mesh
    r = orc.bin_particles([x, y], [a, b], (1, 0), bnd, ny, nx, ALL)
    assert np.array_equal(r["count"], base["count"].T)
    for j in range(2):
        assert same_bits(r["min"][j], base["min"][j].T) and same_bits(r["max"][j], base["max"][j].T)
    # a 1x1 mesh is the global reduction over the inside particles
    r = orc.bin_particles([x, y], [a, b], (0, 1), bnd, 1, 1, ALL)
    keep = (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)
    assert r["count"][0, 0] == keep.sum()
    for j, v in enumerate([a, b]):
        assert r["min"][j][0, 0] == v[keep].min() and r["max"][j][0, 0] == v[keep].max()
        assert math.isclose(r["sum"][j][0, 0], math.fsum(v[keep]), rel_tol=1e-12)


def pin_lattice(orc):
    """One particle at every bin centre, value = its flat index: count 1 and
    sum = min = max = avg = that value everywhere."""
    nx, ny = 13, 7
    lo_x, hi_x, lo_y, hi_y = -1.0, 2.0, 0.5, 4.0
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny))
    x = lo_x + (ix.ravel() + 0.5) * (hi_x - lo_x) / nx
    y = lo_y + (iy.ravel() + 0.5) * (hi_y - lo_y) / ny
    v = (iy * nx + ix).ravel().astype(np.float64) - 40.0
    r = orc.bin_particles([x, y], [v], (0, 1), (lo_x, hi_x, lo_y, hi_y), nx, ny, ALL)
    assert np.array_equal(r["count"], np.ones((ny, nx), np.int64))
    want = v.reshape(ny, nx)
    for key in ("sum", "min", "max", "avg"):
        assert np.array_equal(r[key][0], want), key


def pin_signed_zero_order(orc):
    """min/max follow totalOrder: -0 < +0, regardless of arrival order."""
    x = np.array([0.1, 0.2, 0.3, 0.4])
    y = np.array([0.1, 0.1, 0.1, 0.1])
    for vals in ([0.0, -0.0, 0.0, -0.0], [-0.0, 0.0, -0.0, 0.0], [0.0, 0.0, 0.0, -0.0]):
        r = orc.bin_particles([x, y], [np.array(vals)], (0, 1), (0.0, 1.0, 0.0, 1.0), 1, 1, ALL)
        assert np.signbit(r["min"][0][0, 0]) and not np.signbit(r["max"][0][0, 0])
    r = orc.bin_particles([x, y], [np.array([0.0, 0.0, 0.0, 0.0])], (0, 1), (0.0, 1.0, 0.0, 1.0), 1, 1, ALL)
    assert not np.signbit(r["min"][0][0, 0])


def pin_f32_columns(orc):
    """f32 coordinates and attributes are widened exactly: the result equals
    the one from the same values given as f64."""
    rng = np.random.default_rng(3)
    n = 5000
    x = rng.random(n, dtype=np.float32)
    y = rng.random(n, dtype=np.float32)
    a = rng.standard_normal(n, dtype=np.float32)
    r32 = orc.bin_particles([x, y], [a], (0, 1), (0.0, 1.0, 0.0, 1.0), 16, 16, ALL)
    r64 = orc.bin_particles([x.astype(np.float64), y.astype(np.float64)], [a.astype(np.float64)],
                            (0, 1), (0.0, 1.0, 0.0, 1.0), 16, 16, ALL)
    assert np.array_equal(r32["count"], r64["count"])
    assert same_bits(r32["min"][0], r64["min"][0]) and same_bits(r32["sum"][0], r64["sum"][0])


ALL_PINS = [pin_golden, pin_bruteforce_random, pin_bruteforce_edges, pin_general_bounds_near_edges,
            pin_scipy, pin_invariants, pin_metamorphic, pin_lattice, pin_signed_zero_order,
            pin_f32_columns]


def pin_auto_bounds(orc):
    """Bounds from the data: brute force agreement, extremes in the first and
    last cells, non-finite coordinates ignored, zero-extent axes."""
    rng = np.random.default_rng(21)
    n = 700
    x = rng.uniform(-3, 5, n)
    y = rng.uniform(2, 2.5, n)
    x[:3] = [np.nan, np.inf, -np.inf]
    y[10] = np.nan
    a = rng.standard_normal(n)
    r = orc.bin_particles([x, y], [a], (0, 1), None, 16, 8, ALL)
    bf = orc_bruteforce([x, y], [a], (0, 1), None, 16, 8)
    assert np.array_equal(r["count"], bf["count"])
    assert same_bits(r["min"][0], bf["min"][0]) and same_bits(r["max"][0], bf["max"][0])
    fin = np.isfinite(x) & np.isfinite(y)
    assert r["inside"] == int(fin.sum())
    xf, yf = x[np.isfinite(x)], y[np.isfinite(y)]
    ix_min = int(np.argmin(np.where(np.isfinite(x), x, np.inf)))
    ix_max = int(np.argmax(np.where(np.isfinite(x), x, -np.inf)))
    bnd = (xf.min(), xf.max(), yf.min(), yf.max())
    assert orc.auto_bounds([x, y], (0, 1)) == bnd
    r2 = orc.bin_particles([x, y], [a], (0, 1), bnd, 16, 8, ALL)
    assert np.array_equal(r["count"], r2["count"])
    # the extreme particles sit in the first and the last column
    inside, idx = orc.axis_index(x, bnd[0], bnd[1], 16)
    assert idx[ix_min] == 0 and idx[ix_max] == 15 and inside[ix_min] and inside[ix_max]
    # zero extent: all finite particles in the first cell of that axis
    xc = np.full(50, 0.75)
    yc = rng.uniform(0, 1, 50)
    r = orc.bin_particles([xc, yc], [np.ones(50)], (0, 1), None, 4, 5, ALL)
    assert r["count"][:, 0].sum() == 50 and r["count"][:, 1:].sum() == 0
    # no finite value: nothing inside
    r = orc.bin_particles([np.full(5, np.nan), np.ones(5)], [np.ones(5)], (0, 1), None, 3, 3, ALL)
    assert r["inside"] == 0 and r["count"].sum() == 0
    # extents with no finite binary64 scale count as zero extent: data
    # spanning more than the largest double (hi - lo overflows), and a
    # subnormal extent (nbins / (hi - lo) overflows); every finite particle
    # is inside, in the first cell of that axis, on both oracle paths.
    big = np.array([-1.5e308, 1.5e308, 0.0, 1e300, -1e300, np.inf])
    tiny = np.array([0.0, 5e-324, 1e-323, 5e-324, 0.0, np.nan])
    yv = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6])
    for col in (big, tiny):
        for res in (orc.bin_particles([col, yv], [yv], (0, 1), None, 8, 2, ALL),
                    orc_bruteforce([col, yv], [yv], (0, 1), None, 8, 2)):
            assert res["inside"] == 5 and res["count"][:, 0].sum() == 5 and res["count"][:, 1:].sum() == 0
        inside, idx = orc.axis_index(col, *orc.auto_bounds([col], (0,)), 8)
        assert inside.sum() == 5 and np.all(idx[inside] == 0)


ALL_PINS.append(pin_auto_bounds)


# --------------------------------------------------------------------------
# One to three axes (Section 4.2: any subset of the variables spans the mesh).
# --------------------------------------------------------------------------

def orc_bruteforce_nd(coords, attrs, axes, bounds, dims):
    from oracle import binning_oracle as real
    return real.bin_particles_nd_bruteforce(coords, attrs, axes, bounds, dims)


def _same_result(r, ref, nattr, sum_rel=1e-13, what=""):
    assert r["inside"] == ref["inside"], what
    assert r["count"].shape == ref["count"].shape, what
    assert np.array_equal(r["count"], ref["count"]), what
    for j in range(nattr):
        assert np.all(np.abs(r["sum"][j] - ref["sum"][j]) <= sum_rel * ref["abs_sum"][j]), (what, "sum")
        assert same_bits(r["min"][j], ref["min"][j]), (what, "min")
        assert same_bits(r["max"][j], ref["max"][j]), (what, "max")
        cnt = ref["count"]
        ok = np.where(cnt == 0, np.isnan(r["avg"][j]),
                      np.abs(r["avg"][j] - ref["avg"][j]) <= sum_rel * ref["abs_sum"][j] / np.maximum(cnt, 1))
        assert np.all(ok), (what, "avg")


def pin_nd_golden(orc):
    with open(os.path.join(HERE, "golden", "hand_cases_nd.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        cols = [np.array([_num(v) for v in case[c]]) for c in ("x", "y", "z") if c in case]
        attrs = [np.array([_num(v) for v in case["a"]])]
        r = orc.bin_particles_nd(cols, attrs, tuple(case["axes"]), tuple(case["bounds"]), tuple(case["dims"]), ALL)
        name = case["name"]
        assert r["inside"] == case["inside"], name
        assert r["count"].shape == tuple(reversed(case["dims"])), name
        assert np.array_equal(r["count"], np.array(case["count"])), name
        assert np.array_equal(r["sum"][0], _arr(case["sum"][0])), (name, "sum")
        for key in ("min", "max", "avg"):
            assert same_bits(r[key][0], _arr(case[key][0])), (name, key)


def pin_nd_bruteforce(orc):
    """Random particles on dyadic 1-D and 3-D meshes of unequal sides (so a
    transposed layout changes the shape or the cell), plus given-bounds and
    data-bounds cases, against the per-cell rational brute force."""
    rng = np.random.default_rng(31)
    n = 700
    cols = [rng.uniform(-0.1, 1.1, n), rng.uniform(-2.2, 2.2, n), rng.uniform(0.2, 0.8, n), rng.standard_normal(n)]
    cols[0][:4] = [np.nan, 1.0, 0.0, np.inf]
    cols[2][4:6] = [0.25, 0.75]
    a = rng.standard_normal(n) * 3
    m = rng.lognormal(0, 1, n)
    for axes, bounds, dims in [((0, 1, 2), (0.0, 1.0, -2.0, 2.0, 0.25, 0.75), (8, 4, 2)),
                               ((2, 0, 1), (0.25, 0.75, 0.0, 1.0, -2.0, 2.0), (2, 16, 4)),
                               ((1, 2, 0), (-2.0, 2.0, 0.25, 0.75, 0.0, 1.0), (1, 1, 1)),
                               ((0, 1, 2), (0.0, 1.0, -2.0, 2.0, 0.25, 0.75), (3, 5, 7)),
                               ((1,), (-2.0, 2.0), (16,)),
                               ((2,), (0.25, 0.75), (1,)),
                               ((0, 3), (0.0, 1.0, -1.0, 1.0), (4, 8))]:
        r = orc.bin_particles_nd(cols, [a, m], axes, bounds, dims, ALL)
        _same_result(r, orc_bruteforce_nd(cols, [a, m], axes, bounds, dims), 2, what=str((axes, dims)))
    for axes, dims in [((0, 1, 3), (4, 3, 5)), ((3,), (9,))]:
        r = orc.bin_particles_nd(cols, [a], axes, None, dims, ALL)
        _same_result(r, orc_bruteforce_nd(cols, [a], axes, None, dims), 1, what=f"auto {axes}")


def pin_nd_libraries(orc):
    """NumPy histogram/histogramdd and SciPy binned_statistic(_dd) on dyadic
    meshes (count, sum, min, max, mean); their arrays are indexed [axis 0]
    [axis 1][axis 2], ours the reverse."""
    from scipy.stats import binned_statistic, binned_statistic_dd
    rng = np.random.default_rng(41)
    n = 20000
    x, y, z = rng.random(n), rng.random(n) * 2 - 1, rng.random(n) * 4
    x[:40] = 1.0
    y[40:80] = 1.0
    z[80:120] = 4.0
    a = rng.standard_normal(n) + 0.25
    # one axis
    r = orc.bin_particles_nd([x, y, z], [a], (2,), (0.0, 4.0), (32,), ALL)
    e = np.linspace(0, 4, 33)
    assert np.array_equal(r["count"], np.histogram(z, bins=e)[0])
    full = r["count"] > 0
    for stat, key in (("sum", "sum"), ("mean", "avg")):
        ref = binned_statistic(z, a, stat, bins=e).statistic
        assert np.allclose(r[key][0][full], ref[full], rtol=1e-12, atol=1e-12), key
    for stat in ("min", "max"):
        assert np.array_equal(r[stat][0][full], binned_statistic(z, a, stat, bins=e).statistic[full]), stat
    # three axes
    dims = (8, 4, 16)
    edges = [np.linspace(0, 1, 9), np.linspace(-1, 1, 5), np.linspace(0, 4, 17)]
    r = orc.bin_particles_nd([x, y, z], [a], (0, 1, 2), (0.0, 1.0, -1.0, 1.0, 0.0, 4.0), dims, ALL)
    h, _ = np.histogramdd(np.stack([x, y, z], axis=1), bins=edges)
    assert np.array_equal(r["count"], h.transpose(2, 1, 0).astype(np.int64))
    full = r["count"] > 0
    for stat, key in (("sum", "sum"), ("mean", "avg"), ("min", "min"), ("max", "max")):
        ref = binned_statistic_dd(np.stack([x, y, z], axis=1), a, stat, bins=edges).statistic.transpose(2, 1, 0)
        if key in ("min", "max"):
            assert np.array_equal(r[key][0][full], ref[full]), key
        else:
            assert np.allclose(r[key][0][full], ref[full], rtol=1e-12, atol=1e-12), key


def pin_nd_reductions(orc):
    """Marginals: summing a 3-D result over an axis gives the 2-D result over
    the other two axes (when every particle is inside the summed axis's
    bounds), a single z bin gives the 2-D mesh, and two axes through
    bin_particles_nd give bin_particles bit for bit."""
    rng = np.random.default_rng(43)
    n = 40000
    x, y, z = rng.uniform(-0.1, 1.1, n), rng.uniform(0, 3, n), rng.uniform(-1, 1, n)
    a = rng.standard_normal(n)
    b3 = (0.0, 1.0, 0.0, 3.0, -1.0, 1.0)
    r3 = orc.bin_particles_nd([x, y, z], [a], (0, 1, 2), b3, (10, 6, 5), ALL)
    r2 = orc.bin_particles([x, y, z], [a], (0, 1), b3[:4], 10, 6, ALL)
    assert np.array_equal(r3["count"].sum(axis=0), r2["count"])
    assert np.allclose(r3["sum"][0].sum(axis=0), r2["sum"][0], rtol=1e-12, atol=1e-12)
    mn = np.min(np.where(r3["count"] > 0, r3["min"][0], np.inf), axis=0)
    assert np.array_equal(mn[r2["count"] > 0], r2["min"][0][r2["count"] > 0])
    rx = orc.bin_particles_nd([x, y, z], [a], (2, 1), (-1.0, 1.0, 0.0, 3.0), (5, 6), ALL)
    ins_x = (x >= 0) & (x <= 1)
    rxz = orc.bin_particles_nd([x[ins_x], y[ins_x], z[ins_x]], [a[ins_x]], (2, 1), (-1.0, 1.0, 0.0, 3.0), (5, 6), ALL)
    assert np.array_equal(r3["count"].sum(axis=2), rxz["count"].T)
    assert rx["inside"] == n
    r1 = orc.bin_particles_nd([x, y, z], [a], (0, 1, 2), b3, (10, 6, 1), ALL)
    assert r1["count"].shape == (1, 6, 10)
    for key in ("count",):
        assert np.array_equal(r1[key][0], r2[key])
    for key in ("sum", "min", "max", "avg"):
        assert same_bits(r1[key][0][0], r2[key][0]), key
    rnd = orc.bin_particles_nd([x, y, z], [a], (1, 0), (0.0, 3.0, 0.0, 1.0), (7, 9), ALL)
    r2b = orc.bin_particles([x, y, z], [a], (1, 0), (0.0, 3.0, 0.0, 1.0), 7, 9, ALL)
    assert np.array_equal(rnd["count"], r2b["count"])
    for key in ("sum", "min", "max", "avg"):
        assert same_bits(rnd[key][0], r2b[key][0]), key


def pin_nd_lattice(orc):
    """One particle at every cell centre of a 3-D mesh with non-dyadic bounds,
    valued by its cell's position in C order over [nz][ny][nx], and a line of
    cell centres in 1-D."""
    nx, ny, nz = 5, 3, 4
    lo = (-1.0, 0.5, 10.0)
    hi = (2.0, 4.0, 10.7)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = lo[0] + (ix.ravel() + 0.5) * (hi[0] - lo[0]) / nx
    y = lo[1] + (iy.ravel() + 0.5) * (hi[1] - lo[1]) / ny
    z = lo[2] + (iz.ravel() + 0.5) * (hi[2] - lo[2]) / nz
    v = np.arange(nx * ny * nz, dtype=np.float64) * 1.5 - 7.0
    perm = np.random.default_rng(2).permutation(v.size)
    r = orc.bin_particles_nd([x[perm], y[perm], z[perm]], [v[perm]], (0, 1, 2),
                             (lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]), (nx, ny, nz), ALL)
    assert np.array_equal(r["count"], np.ones((nz, ny, nx), np.int64))
    for key in ("sum", "min", "max", "avg"):
        assert np.array_equal(r[key][0], v.reshape(nz, ny, nx)), key
    w = np.arange(7, dtype=np.float64)
    r = orc.bin_particles_nd([w * 0.5 + 0.25], [w + 1], (0,), (0.0, 3.5), (7,), ALL)
    assert np.array_equal(r["count"], np.ones(7, np.int64)) and np.array_equal(r["sum"][0], w + 1)


ALL_PINS += [pin_nd_golden, pin_nd_bruteforce, pin_nd_libraries, pin_nd_reductions, pin_nd_lattice]
