"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  count/min/max bit-exact; sum/avg within 1e-5 * sum|a|
per bin (default, compensated FP32 and FP64 modes), or the sequential FP32
error bound for the plain FP32 mode.  Every strategy (global atomics, whole
grid in LDS, partition by tile) is run on the cases it can take."""
import sys

import numpy as np
import pytest

from paper_2310_02926_amd import synth
from tests import gpu_check as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _reset_plan():
    from paper_2310_02926_amd import binding as B
    B.bin_set_plan_override(-1, 0, 0)
    yield
    B.bin_set_plan_override(-1, 0, 0)


def _bin(ws, strategy=-1, ops=None, grid=0, block=0, **kw):
    from paper_2310_02926_amd import binding as B
    B.bin_set_plan_override(strategy, block, grid)
    try:
        return G.run_gpu(ws, ops=ops, **kw)
    finally:
        B.bin_set_plan_override(-1, 0, 0)


STRATS = [pytest.param(-1, id="auto"), pytest.param(0, id="global"), pytest.param(1, id="lds"),
          pytest.param(2, id="part")]
PRECS = ["default", "comp", "plain", "f64"]


def _flag(prec):
    from paper_2310_02926_amd import binding as B
    return {"default": 0, "comp": B.PREC_COMP, "plain": B.PREC_PLAIN, "f64": B.PREC_F64}[prec]


@pytest.mark.parametrize("strategy", STRATS)
def test_uniform_f64_65536_64x64(strategy):
    _case(f"uniform f64 n=65536 64x64 strategy={strategy}")
    ws = synth.uniform_f64(65536, seed=0)
    ref = G.oracle(ws)
    got = _bin(ws, strategy)
    G.assert_parity(got, ref, ws.ops, rel=1e-12, what="uniform_f64")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("side,strategy", [(1024, -1), (1024, 0), (32, 1), (32, 2), (48, -1), (200, 2)])
def test_gmm_f32_k4(side, strategy, prec):
    from paper_2310_02926_amd import binding as B
    _case(f"gmm f32 n=2^20+77 side={side} k=4 prec={prec} strategy={strategy}")
    ws = synth.gmm_f32(n=(1 << 20) + 77, seed=1, nx=side, ny=side, k=4)
    ref = G.oracle(ws)
    got = _bin(ws, strategy, ops=B.OPS_ALL | _flag(prec))
    G.assert_parity(got, ref, B.OPS_ALL, plain=(prec == "plain"), what=f"gmm side={side} {prec}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("side,strategy", [(2048, -1), (2048, 0), (64, 1), (64, 2), (512, 2)])
def test_hotspot_f32(side, strategy, prec):
    from paper_2310_02926_amd import binding as B
    _case(f"hotspot f32 n=2^22 side={side} prec={prec} strategy={strategy}")
    ws = synth.hotspot_f32(n=1 << 22, seed=2, side=side)
    ref = G.oracle(ws)
    got = _bin(ws, strategy, ops=B.OPS_ALL | _flag(prec))
    G.assert_parity(got, ref, B.OPS_ALL, plain=(prec == "plain"), what=f"hotspot side={side} {prec}")


def test_partition_split_tiles_clustered():
    """A tile holding far more than the split length is binned by several
    work items whose partials are merged."""
    from paper_2310_02926_amd import binding as B
    _case("partition with split tiles")
    rng = np.random.default_rng(12)
    n = 3_000_000
    x = np.where(rng.random(n) < 0.8, rng.normal(0.5, 0.003, n), rng.random(n)).astype(np.float32)
    y = np.where(rng.random(n) < 0.8, rng.normal(0.5, 0.003, n), rng.random(n)).astype(np.float32)
    ws = synth.Workload([x, y], [rng.lognormal(0, 1, n).astype(np.float32), rng.standard_normal(n).astype(np.float32)],
                        nx=1024, ny=1024)
    for prec in PRECS:
        got = _bin(ws, 2, ops=B.OPS_ALL | _flag(prec))
        G.assert_parity(got, G.oracle(ws), B.OPS_ALL, plain=(prec == "plain"), what=f"split {prec}")


@pytest.mark.parametrize("split_len", [1024, 5000, 65536])
def test_partition_forced_split_lengths(split_len):
    """Short split lengths: most tiles are binned by many items (each a
    range of whole workgroup slices) and merged; a contiguous hot block puts
    most particles into a handful of tiles."""
    from paper_2310_02926_amd import binding as B
    _case(f"partition split_len={split_len}")
    ws = synth.hotspot_f32(n=2_000_000, seed=3, side=512, contiguous=True)
    ref = G.oracle(ws)
    B.bin_set_tuning(B.TUNE_SPLIT_LEN, split_len)
    B.bin_set_tuning(B.TUNE_PART_WG, 700)
    try:
        got = _bin(ws, 2)
    finally:
        B.reset_tuning()
    G.assert_parity(got, ref, 31, what=f"split_len={split_len}")


def _quad_cases():
    rng = np.random.default_rng(77)
    n = 1_500_001  # ragged: the last slice and sub-chunk are partial
    x, y = rng.random(n), rng.random(n)
    yield "hotspot k=1", synth.hotspot_f32(n=2_000_000, seed=5, side=512, contiguous=True), 0
    yield "gmm k=4", synth.gmm_f32(n=1_000_000, seed=6, nx=1024, ny=1024, k=4), 0
    yield "f64 attrs k=2", _ws([x.astype(np.float32), y.astype(np.float32)],
                               [rng.standard_normal(n), rng.lognormal(0, 1, n)], 700, 900), 0
    yield "f64 coords count only", _ws([x, y], [], 2048, 1000, ops=1), 0
    # more attributes than one load round trip holds (4 f32, 2 f64)
    yield "f32 attrs k=9", _ws([x.astype(np.float32), y.astype(np.float32)],
                               [rng.standard_normal(n).astype(np.float32) for _ in range(9)], 300, 200), 0
    yield "f64 attrs k=5", _ws([x.astype(np.float32), y.astype(np.float32)],
                               [rng.lognormal(0, 1, n) for _ in range(5)], 300, 200), 0
    e = synth.edge_points(0.0, 1.0, 1024, np.float32)
    yield "edges", _ws([rng.choice(e, n), rng.choice(e, n)], [rng.standard_normal(n).astype(np.float32)],
                       1024, 1024), 0
    yield "sparse tiles (runs of 1-3 records)", _ws([x.astype(np.float32) * 0.999, y.astype(np.float32)],
                                                   [rng.standard_normal(n).astype(np.float32)], 4096, 4096), 0
    yield "unaligned columns", _ws([x.astype(np.float32), y.astype(np.float32)],
                                   [rng.standard_normal(n).astype(np.float32)], 1500, 1500), 1


@pytest.mark.parametrize("quads", [1, 2], ids=["records", "quads"])
def test_partition_record_and_quad_gathers(quads):
    """Both gathers of the tile binning - record by record, and whole quads
    of 4 records (each tile's run padded with empty records) - on the cases
    the planner would send to either: one or several attributes (more than
    one load round trip holds), f64 attributes and coordinates, count only, bin edges, sparse tiles with
    runs of a few records, a ragged size and unaligned columns."""
    from paper_2310_02926_amd import binding as B
    for name, ws, shift in _quad_cases():
        _case(f"partition gather quads={quads}: {name}")
        ref = G.oracle(ws)
        coords, attrs = G.to_device(ws)
        if shift:  # views at an element offset: no 16-byte loads
            coords = [torch.cat([c[:1], c])[1:] for c in coords]
            attrs = [torch.cat([a[:1], a])[1:] for a in attrs]
        B.bin_set_tuning(B.TUNE_QUADS, quads)
        try:
            got = _bin(ws, 2, coords=coords, attrs=attrs)
            out = B.alloc_outputs(attrs, ws.nx, ws.ny, ws.ops, "cuda")
            req, keep = B.request(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops, out)
            plan = B.bin_describe_plan(req)
        finally:
            B.reset_tuning()
        assert plan.startswith("partition") and f"quads={quads - 1}" in plan, plan
        G.assert_parity(got, ref, ws.ops, what=f"quads={quads} {name}")


def _ws(coords, attrs, nx, ny, bounds=(0.0, 1.0, 0.0, 1.0), axes=(0, 1), ops=31):
    return synth.Workload([np.ascontiguousarray(c) for c in coords], [np.ascontiguousarray(a) for a in attrs],
                          axes=axes, bounds=bounds, nx=nx, ny=ny, ops=ops)


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000003])
def test_ragged_and_empty_sizes(n, strategy):
    _case(f"ragged n={n} strategy={strategy}")
    rng = np.random.default_rng(n)
    ws = _ws([rng.uniform(-0.1, 1.1, n).astype(np.float32), rng.uniform(-0.1, 1.1, n).astype(np.float32)],
             [rng.standard_normal(n).astype(np.float32), rng.lognormal(0, 1, n).astype(np.float32)], 40, 24)
    G.assert_parity(_bin(ws, strategy), G.oracle(ws), 31, what=f"n={n}")


@pytest.mark.parametrize("strategy", STRATS)
def test_edges_nan_inf_and_closed_upper_edge(strategy):
    _case(f"edge points strategy={strategy}")
    for dt in (np.float32, np.float64):
        for (nx, lo, hi) in [(64, 0.0, 1.0), (10, -0.3, 0.7), (7, 1.0, 1.1), (3000, 0.0, 1.0)]:
            e = synth.edge_points(lo, hi, nx, dt)
            m = e.size
            xs = np.concatenate([e, np.full(m, (lo + hi) / 2, dt)])
            ys = np.concatenate([np.full(m, 0.5, dt), np.linspace(-0.2, 1.2, m).astype(dt)])
            a = np.arange(2 * m, dtype=np.float32) - m
            ws = _ws([xs, ys], [a], nx, 5, bounds=(lo, hi, 0.0, 1.0))
            G.assert_parity(_bin(ws, strategy), G.oracle(ws), 31, what=f"edges {dt.__name__} nx={nx}")


@pytest.mark.parametrize("strategy", STRATS)
def test_all_outside_gives_empty_bins(strategy):
    _case(f"all outside strategy={strategy}")
    n = 5000
    ws = _ws([np.full(n, 2.0, np.float32), np.linspace(0, 1, n).astype(np.float32)],
             [np.ones(n, np.float32)], 16, 16)
    got = _bin(ws, strategy)
    assert got["count"].sum() == 0
    assert np.all(np.isposinf(got["min"][0])) and np.all(np.isneginf(got["max"][0]))
    assert np.all(got["sum"][0] == 0) and np.all(np.isnan(got["avg"][0]))


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 300), (4096, 1), (3, 5), (70000, 3)])
def test_degenerate_grids(nx, ny, strategy):
    _case(f"grid {nx}x{ny} strategy={strategy}")
    rng = np.random.default_rng(nx * 7 + ny)
    n = 200_000
    ws = _ws([rng.random(n), rng.random(n)], [rng.standard_normal(n), rng.lognormal(0, 1, n)], nx, ny)
    G.assert_parity(_bin(ws, strategy), G.oracle(ws), 31, rel=1e-12, what=f"{nx}x{ny}")


@pytest.mark.parametrize("strategy", STRATS)
def test_axes_from_wider_table_and_mixed_dtypes(strategy):
    _case(f"axes (2,0) of xyz, f64 coords, f32 attrs, strategy={strategy}")
    rng = np.random.default_rng(9)
    n = 300_001
    x, y, z = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-2, 2, n)
    attrs = [rng.standard_normal(n).astype(np.float32) for _ in range(3)]
    ws = _ws([x, y, z], attrs, 50, 20, bounds=(-2.0, 2.0, -1.0, 1.0), axes=(2, 0))
    G.assert_parity(_bin(ws, strategy), G.oracle(ws), 31, what="xz-plane")


@pytest.mark.parametrize("ops", [1, 2, 4, 8, 16, 1 | 4, 2 | 8, 16 | 4, 31])
@pytest.mark.parametrize("strategy", STRATS)
def test_op_subsets(ops, strategy):
    _case(f"ops={ops} strategy={strategy}")
    ws = synth.gmm_f32(n=400_000, seed=5, nx=40, ny=40, k=2)
    got = _bin(ws, strategy, ops=ops)
    from paper_2310_02926_amd import binding as B
    for key, bit in (("count", B.COUNT), ("sum", B.SUM), ("min", B.MIN), ("max", B.MAX), ("avg", B.AVG)):
        assert (key in got) == bool(ops & bit)
    G.assert_parity(got, G.oracle(ws), ops, what=f"ops={ops}")


@pytest.mark.parametrize("strategy", STRATS)
def test_count_only_without_attributes(strategy):
    _case(f"count only, k=0, strategy={strategy}")
    rng = np.random.default_rng(4)
    n = 123_457
    ws = _ws([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)], [], 300, 300, ops=1)
    got = _bin(ws, strategy, ops=1)
    assert np.array_equal(got["count"], G.oracle(ws)["count"])


@pytest.mark.parametrize("strategy", STRATS)
def test_signed_zeros_min_max(strategy):
    _case(f"signed zeros strategy={strategy}")
    n = 4096
    x = (np.arange(n) % 4 + 0.5).astype(np.float32) / 4
    y = np.full(n, 0.5, np.float32)
    a = np.where(np.arange(n) % 3 == 0, -0.0, 0.0).astype(np.float32)
    ws = _ws([x, y], [a], 4, 1)
    got = _bin(ws, strategy)
    assert np.all(np.signbit(got["min"][0])) and not np.any(np.signbit(got["max"][0]))
    G.assert_parity(got, G.oracle(ws), 31, what="zeros")


@pytest.mark.parametrize("strategy", STRATS)
def test_sixteen_attributes(strategy):
    _case(f"16 attributes strategy={strategy}")
    rng = np.random.default_rng(16)
    n = 100_000
    ws = _ws([rng.random(n, dtype=np.float32), rng.random(n, dtype=np.float32)],
             [rng.standard_normal(n).astype(np.float32) for _ in range(16)], 33, 17)
    G.assert_parity(_bin(ws, strategy), G.oracle(ws), 31, what="k=16")


def test_exact_ops_identical_across_launch_shapes():
    """Races cannot change count/min/max: identical over launch shapes."""
    _case("determinism over launch shapes")
    ws = synth.hotspot_f32(n=1 << 21, seed=3, side=256)
    coords, attrs = G.to_device(ws)
    base = _bin(ws, 0, coords=coords, attrs=attrs)
    for strategy, grid, block in [(0, 7, 64), (0, 1000, 256), (0, 4096, 1024), (2, 3, 0), (2, 300, 0),
                                  (2, 1, 0), (1, 3, 256), (-1, 0, 0)]:
        got = _bin(ws, strategy, grid=grid, block=block, coords=coords, attrs=attrs)
        assert np.array_equal(got["count"], base["count"])
        assert np.array_equal(got["min"][0].view(np.int32), base["min"][0].view(np.int32))
        assert np.array_equal(got["max"][0].view(np.int32), base["max"][0].view(np.int32))
        assert np.allclose(got["sum"][0], base["sum"][0], rtol=1e-9, atol=0)


def test_side_stream_and_reuse_of_outputs():
    _case("side stream, outputs overwritten")
    from paper_2310_02926_amd import binding as B
    ws = synth.gmm_f32(n=300_000, seed=8, nx=128, ny=128, k=1)
    coords, attrs = G.to_device(ws)
    s = torch.cuda.Stream()
    out = B.alloc_outputs(attrs, 128, 128, 31, coords[0].device)
    for _ in range(3):  # outputs are overwritten, not accumulated
        B.bin_particles(coords, attrs, ws.n, (0, 1), ws.bounds, 128, 128, 31, out, stream=s)
    s.synchronize()
    got = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
    for key in ("sum", "min", "max", "avg"):
        got[key] = [t.cpu().numpy() for t in out[key]]
    G.assert_parity(got, G.oracle(ws), 31, what="side stream")
    assert B.bin_stream_status(s) == B.BIN_OK


def test_timing_report_names_kernels():
    from paper_2310_02926_amd import binding as B
    ws = synth.hotspot_f32(n=1 << 20, seed=4, side=1024)
    coords, attrs = G.to_device(ws)
    B.bin_timing_enable(True)
    G.run_gpu(ws, coords=coords, attrs=attrs)
    B.bin_timing_enable(False)
    rep = B.bin_timing_report()
    assert "part_scatter_kernel" in rep and "part_bin_kernel" in rep, rep
    n, ms = B.bin_timing_read()
    assert n >= 1 and ms > 0 and abs(ms - max(v[1] for v in rep.values())) < 1e-5


def test_single_hip_runtime_on_gpu():
    from paper_2310_02926_amd import binding as B
    B.lib()
    torch.zeros(1, device="cuda")
    libs = {l.split()[-1] for l in open("/proc/self/maps").read().splitlines() if "libamdhip64" in l}
    assert len(libs) == 1, libs


def _run_auto(ws, strategy=-1, ops=31):
    from paper_2310_02926_amd import binding as B
    coords, attrs = G.to_device(ws)
    B.bin_set_plan_override(strategy, 0, 0)
    try:
        out = B.bin_particles_alloc(coords, attrs, ws.axes, None, ws.nx, ws.ny, ops)
    finally:
        B.bin_set_plan_override(-1, 0, 0)
    torch.cuda.synchronize()
    res = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


@pytest.mark.parametrize("strategy", STRATS)
def test_auto_bounds(strategy):
    """Bounds from the data (Section 4.2): the oracle's reading R9."""
    _case(f"auto bounds strategy={strategy}")
    from oracle import binning_oracle as orc
    rng = np.random.default_rng(31)
    n = 500_003
    x = rng.normal(3.0, 2.0, n).astype(np.float32)
    y = rng.uniform(-7, -2, n).astype(np.float32)
    x[:5] = [np.nan, np.inf, -np.inf, np.nan, 0.0]
    y[7] = np.inf
    a = rng.lognormal(0, 1, n).astype(np.float32)
    for (nx, ny) in [(64, 64), (1000, 900)]:
        ws = _ws([x, y], [a], nx, ny)
        ref = orc.bin_particles(ws.coords, ws.attrs, (0, 1), None, nx, ny)
        G.assert_parity(_run_auto(ws, strategy), ref, 31, what=f"auto {nx}x{ny}")


@pytest.mark.parametrize("strategy", STRATS)
def test_auto_bounds_degenerate(strategy):
    _case(f"auto bounds degenerate strategy={strategy}")
    from oracle import binning_oracle as orc
    rng = np.random.default_rng(32)
    n = 10_000
    # zero-extent x axis
    ws = _ws([np.full(n, 0.25), rng.random(n)], [rng.standard_normal(n)], 8, 8)
    ref = orc.bin_particles(ws.coords, ws.attrs, (0, 1), None, 8, 8)
    got = _run_auto(ws, strategy)
    assert got["count"][:, 1:].sum() == 0 and got["count"].sum() == n
    G.assert_parity(got, ref, 31, rel=1e-12, what="zero extent")
    # no finite coordinate at all
    ws = _ws([np.full(n, np.nan), rng.random(n)], [rng.standard_normal(n)], 8, 8)
    got = _run_auto(ws, strategy)
    assert got["count"].sum() == 0 and np.all(np.isnan(got["avg"][0]))
    # extents with no finite binary64 scale (R9): binary64 data spanning more
    # than the largest double, and a subnormal extent; both count as zero
    # extent, every finite particle in the first column
    big = rng.uniform(-1.0, 1.0, n) * 1.7e308
    big[:2] = [-1.7e308, 1.7e308]
    tiny = rng.integers(0, 4, n).astype(np.float64) * 5e-324
    tiny[3] = np.inf
    for col, what in ((big, "overflowing extent"), (tiny, "subnormal extent")):
        ws = _ws([col, rng.random(n)], [rng.standard_normal(n)], 8, 8)
        ref = orc.bin_particles(ws.coords, ws.attrs, (0, 1), None, 8, 8)
        got = _run_auto(ws, strategy)
        assert got["count"][:, 1:].sum() == 0 and got["count"].sum() == int(np.isfinite(col).sum()), what
        G.assert_parity(got, ref, 31, rel=1e-12, what=what)


@pytest.mark.parametrize("strategy", [pytest.param(1, id="lds"), pytest.param(2, id="part")])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shift", [0, 1, 3])
def test_unaligned_columns_take_the_narrow_load_path(strategy, dtype, shift):
    """Columns that start off a 16-byte boundary (views into larger buffers)
    are read element by element; results equal the aligned case's oracle."""
    from paper_2310_02926_amd import binding as B
    _case(f"unaligned columns shift={shift} dtype={np.dtype(dtype).name} strategy={strategy}")
    rng = np.random.default_rng(100 + shift)
    n = 1_000_037
    side = 64 if strategy == 1 else 1024
    ws = _ws([rng.uniform(-0.05, 1.05, n).astype(dtype), rng.uniform(-0.05, 1.05, n).astype(dtype)],
             [rng.standard_normal(n).astype(np.float32), rng.lognormal(0, 1, n).astype(np.float32)], side, side)
    dev_c, dev_a = G.to_device(ws)
    # the first coordinate column and the second attribute start `shift` elements into their buffers
    xbuf = torch.empty(n + shift, dtype=dev_c[0].dtype, device="cuda")
    xbuf[shift:] = dev_c[0]
    abuf = torch.empty(n + shift, dtype=dev_a[1].dtype, device="cuda")
    abuf[shift:] = dev_a[1]
    coords = [xbuf[shift:], dev_c[1]]
    attrs = [dev_a[0], abuf[shift:]]
    B.bin_set_plan_override(strategy, 0, 0)
    try:
        out = B.alloc_outputs(attrs, ws.nx, ws.ny, 31, "cuda")
        req, keep = B.request(coords, attrs, n, ws.axes, ws.bounds, ws.nx, ws.ny, 31, out)
        desc = B.bin_describe_plan(req)
        assert f"vec={0 if shift else 1}" in desc, desc
        got = G.run_gpu(ws, coords=coords, attrs=attrs)
    finally:
        B.bin_set_plan_override(-1, 0, 0)
    G.assert_parity(got, G.oracle(ws), 31, what=f"unaligned shift={shift}")


def test_plan_without_gpu_matches_device_plan():
    """bin_describe_plan_on with this device's sizes gives the plan the
    library makes on the device (so the planner tests on the CPU test the
    plans that run here)."""
    from paper_2310_02926_amd import binding as B
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    lds = props.shared_memory_per_block
    for (n, side, k) in [(1 << 27, 2048, 1), (1 << 24, 1024, 4), (1 << 24, 128, 1), (1 << 24, 64, 1), (65536, 64, 1),
                         (0xFFFFFFFF, 2048, 1), ((1 << 32) - (1 << 21) + 1, 2048, 1)]:
        coords = [torch.empty(8, device="cuda") for _ in range(2)]
        attrs = [torch.empty(8, device="cuda") for _ in range(k)]
        out = B.alloc_outputs(attrs, side, side, 31, "cuda")
        req, keep = B.request(coords, attrs, n, (0, 1), (0.0, 1.0, 0.0, 1.0), side, side, 31, out)
        assert B.bin_describe_plan(req) == B.bin_describe_plan_on(req, cus, lds, lds), (n, side, k)


def test_prepared_call_repeats_match_oracle():
    """A request marshalled once (binding.Call) and launched several times
    into the same outputs gives the oracle's result each time, as when a
    simulation bins every step."""
    from paper_2310_02926_amd import binding as B
    _case("prepared call, three launches, gmm f32 k=4 512x512")
    ws = synth.gmm_f32(n=300_000, seed=5, nx=512, ny=512, k=4)
    coords, attrs = G.to_device(ws)
    out = B.alloc_outputs(attrs, ws.nx, ws.ny, ws.ops, coords[0].device)
    call = B.Call(coords, attrs, ws.n, ws.axes, ws.bounds, ws.nx, ws.ny, ws.ops, out)
    ref = G.oracle(ws)
    s = torch.cuda.Stream()
    for step in range(3):
        for t in [out["count"]] + [x for key in ("sum", "min", "max", "avg") for x in out.get(key, [])]:
            t.fill_(7)
        torch.cuda.synchronize()
        call.launch(s)
        s.synchronize()
        got = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
        for key in ("sum", "min", "max", "avg"):
            got[key] = [t.cpu().numpy() for t in out[key]]
        G.assert_parity(got, ref, ws.ops, what=f"prepared call launch {step}")
