"""GPU parity of bin_particles_nd (meshes of one, two or three axes) against
the oracle's bin_particles_nd: count/min/max bit-exact, sum/avg within
1e-5 * sum|a| per bin, every strategy on the cases it can take."""
import sys

import numpy as np
import pytest

from oracle import binning_oracle as orc
from paper_2310_02926_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from tests import gpu_check as G  # noqa: E402

STRATS = [pytest.param(-1, id="auto"), pytest.param(0, id="global"), pytest.param(1, id="lds"),
          pytest.param(2, id="part")]


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _reset_plan():
    from paper_2310_02926_amd import binding as B
    B.bin_set_plan_override(-1, 0, 0)
    yield
    B.bin_set_plan_override(-1, 0, 0)


def _run(cols, attrs, axes, bounds, dims, ops=31, strategy=-1, dev_cols=None, dev_attrs=None):
    from paper_2310_02926_amd import binding as B
    dc = dev_cols if dev_cols is not None else [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cols]
    da = dev_attrs if dev_attrs is not None else [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in attrs]
    n = len(cols[0])
    out = B.alloc_outputs_nd(da, dims, ops, "cuda")
    B.bin_set_plan_override(strategy, 0, 0)
    try:
        B.bin_particles_nd(dc, da, n, axes, bounds, dims, ops, out)
        torch.cuda.synchronize()
    finally:
        B.bin_set_plan_override(-1, 0, 0)
    res = {}
    if "count" in out:
        res["count"] = out["count"].cpu().numpy().view(np.uint32).astype(np.int64)
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def _check(cols, attrs, axes, bounds, dims, ops=31, strategy=-1, what="", **kw):
    got = _run(cols, attrs, axes, bounds, dims, ops, strategy, **kw)
    ref = orc.bin_particles_nd(cols, attrs, axes, bounds, dims)
    assert got["count"].shape == tuple(reversed(dims)), what
    G.assert_parity(got, ref, ops, what=what)
    return got, ref


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("dims", [(8, 4, 2), (64, 32, 16), (128, 96, 80), (1, 1, 1), (3, 700, 5)])
@pytest.mark.parametrize("auto", [False, True], ids=["given", "auto"])
def test_three_axes_positions(dims, strategy, auto):
    """Positions of an N-body-like table on a 3-D mesh (n spans several
    tiles and a ragged tail); bounds given or from the data."""
    _case(f"3d positions dims={dims} strategy={strategy} auto={auto}")
    tab = synth.insitu_table(300_001, seed=sum(dims))
    bounds = None if auto else (-1.0, 1.0, -0.75, 0.75, -1.0, 0.5)
    _check(tab.columns, [tab.columns[9], tab.columns[3]], (0, 1, 2), bounds, dims, strategy=strategy,
           what=f"3d {dims}")


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("cdt,adt", [(np.float64, np.float64), (np.float64, np.float32), (np.float32, np.float64)])
def test_three_axes_f64(cdt, adt, strategy):
    _case(f"3d dtypes {cdt.__name__}/{adt.__name__} strategy={strategy}")
    rng = np.random.default_rng(5)
    n = 200_003
    cols = [rng.uniform(-0.1, 1.1, n).astype(cdt) for _ in range(3)]
    attrs = [rng.standard_normal(n).astype(adt), rng.lognormal(0, 1, n).astype(adt)]
    _check(cols, attrs, (2, 0, 1), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), (40, 30, 20), strategy=strategy,
           what="3d f64")


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("nb", [1, 7, 1000, 300_000])
def test_one_axis(nb, strategy):
    """One axis (a velocity component, and the lognormal mass with bounds
    from the data)."""
    _case(f"1d nb={nb} strategy={strategy}")
    tab = synth.insitu_table(250_000, seed=nb)
    _check(tab.columns, [tab.columns[9], tab.columns[0]], (3,), (-4.0, 4.0), (nb,), strategy=strategy,
           what=f"1d {nb}")
    _check(tab.columns, [tab.columns[3]], (9,), None, (nb,), strategy=strategy, what=f"1d auto {nb}")


def test_two_axes_equal_bin_particles():
    from paper_2310_02926_amd import binding as B
    _case("2d through bin_particles_nd")
    tab = synth.insitu_table(100_000, seed=2)
    got, _ = _check(tab.columns, [tab.columns[9]], (4, 5), (-4.0, 4.0, -3.0, 3.0), (50, 60), what="2d")
    cols = [torch.from_numpy(c).cuda() for c in tab.columns]
    out = B.bin_particles_alloc(cols, [cols[9]], (4, 5), (-4.0, 4.0, -3.0, 3.0), 50, 60, 31)
    torch.cuda.synchronize()
    assert np.array_equal(out["count"].cpu().numpy().view(np.uint32).astype(np.int64), got["count"])
    assert np.array_equal(out["min"][0].cpu().numpy(), got["min"][0])


@pytest.mark.parametrize("strategy", STRATS)
def test_three_axes_edges_nan_inf(strategy):
    """Every bin edge of every axis, one-ulp neighbours, NaN and +-Inf, on
    dyadic meshes where the binary64 index is exact."""
    _case(f"3d edges strategy={strategy}")
    rng = np.random.default_rng(8)
    pts = [synth.edge_points(0.0, 1.0, 16, np.float32), synth.edge_points(-2.0, 2.0, 8, np.float32),
           synth.edge_points(0.0, 0.5, 4, np.float32)]
    n = 60_000
    cols = [rng.choice(p, n).astype(np.float32) for p in pts]
    cols[2][:10] = np.nan
    cols[1][10:20] = np.inf
    cols[0][20:30] = -np.inf
    attrs = [rng.standard_normal(n).astype(np.float32)]
    _check(cols, attrs, (0, 1, 2), (0.0, 1.0, -2.0, 2.0, 0.0, 0.5), (16, 8, 4), strategy=strategy, what="edges")


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("n", [0, 1, 3, 1023, 4097])
def test_three_axes_tiny_and_empty(n, strategy):
    _case(f"3d n={n} strategy={strategy}")
    rng = np.random.default_rng(n)
    cols = [rng.random(n).astype(np.float32) for _ in range(3)]
    attrs = [rng.standard_normal(n).astype(np.float32)]
    _check(cols, attrs, (0, 1, 2), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), (5, 6, 7), strategy=strategy, what=f"n={n}")
    if n:
        _check(cols, attrs, (0, 1, 2), None, (5, 6, 7), strategy=strategy, what=f"auto n={n}")


@pytest.mark.parametrize("shift", [1, 3])
def test_three_axes_unaligned_columns(shift):
    """Axis columns that are views at an element offset: the fold takes its
    narrow load path."""
    _case(f"3d unaligned shift={shift}")
    rng = np.random.default_rng(shift)
    n = 100_000
    big = [rng.random(n + shift).astype(np.float32) for _ in range(3)]
    a = rng.standard_normal(n + shift).astype(np.float32)
    dev = [torch.from_numpy(c).cuda()[shift:] for c in big]
    cols = [c[shift:] for c in big]
    da = [torch.from_numpy(a).cuda()[shift:]]
    _check(cols, [a[shift:]], (0, 1, 2), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), (20, 24, 28), what="unaligned",
           dev_cols=dev, dev_attrs=da)


def test_three_axes_degenerate_auto_bounds():
    """Bounds from the data with a zero-extent axis (all in its first cell)
    and with an axis that has no finite value (nothing inside)."""
    _case("3d auto degenerate")
    rng = np.random.default_rng(9)
    n = 50_000
    x, y = rng.random(n).astype(np.float32), rng.random(n).astype(np.float32)
    z = np.full(n, 0.25, np.float32)
    a = [rng.standard_normal(n).astype(np.float32)]
    got, _ = _check([x, y, z], a, (0, 1, 2), None, (8, 8, 4), what="zero extent z")
    assert got["count"][1:].sum() == 0
    z2 = np.full(n, np.nan, np.float32)
    got, _ = _check([x, y, z2], a, (0, 1, 2), None, (8, 8, 4), what="no finite z")
    assert got["count"].sum() == 0


def test_three_axes_large_mesh_sampled():
    """A 256^3 mesh (2^24 bins, the largest folded f32 composite) on 2^22
    particles, checked against the oracle on every bin."""
    _case("3d 256^3")
    tab = synth.insitu_table(1 << 22, seed=12)
    _check(tab.columns, [tab.columns[9]], (0, 1, 2), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), (256, 256, 256),
           ops=31, what="256^3")
