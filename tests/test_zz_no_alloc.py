"""GPU tests of bin_particles_noalloc, the allocation-free variant of
bin_particles: same results as bin_particles (and the oracle) on calls in a
row that reuse its fixed scratch array, with the second call smaller;
requests too large for the array are refused before anything is enqueued;
and the call takes no device memory."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import binning_oracle as orc  # noqa: E402
from paper_2310_02926_amd import binding as B  # noqa: E402
from paper_2310_02926_amd import synth  # noqa: E402
from tests import gpu_check as G  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _ws(n, side, k, seed, bounds=(0.0, 1.0, 0.0, 1.0)):
    rng = np.random.default_rng(seed)
    coords = [rng.uniform(-0.05, 1.05, n).astype(np.float32), rng.uniform(-0.05, 1.05, n).astype(np.float32)]
    attrs = [rng.lognormal(0, 1, n).astype(np.float32)] + [rng.standard_normal(n).astype(np.float32)
                                                          for _ in range(k - 1)]
    return synth.Workload(coords, attrs, axes=(0, 1), bounds=bounds, nx=side, ny=side, ops=B.OPS_ALL)


def _to_np(out):
    res = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
    for key in ("sum", "min", "max", "avg"):
        res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def _run(fn, ws, bounds, stream):
    coords, attrs = G.to_device(ws)
    out = B.alloc_outputs(attrs, ws.nx, ws.ny, B.OPS_ALL, "cuda")
    fn(coords, attrs, ws.n, ws.axes, bounds, ws.nx, ws.ny, B.OPS_ALL, out, stream=stream)
    stream.synchronize()
    return _to_np(out)


def _same_as_plain_call(got, ref):
    """count, min and max identical to bin_particles; sums and averages
    equal up to the rounding order of the binary64 accumulation."""
    assert np.array_equal(got["count"], ref["count"])
    for j in range(len(ref["sum"])):
        for key in ("min", "max"):
            assert np.array_equal(got[key][j].view(np.int32), ref[key][j].view(np.int32)), key
        for key in ("sum", "avg"):
            g, r = got[key][j], ref[key][j]
            assert np.array_equal(np.isnan(g), np.isnan(r)), key
            ok = ~np.isnan(r)
            assert np.all(np.abs(g[ok] - r[ok]) <= 1e-12 * np.maximum(np.abs(r[ok]), 1e-300)), key


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large_then_small"])
def test_noalloc_matches_bin_particles_on_calls_in_a_row(order):
    """Calls in a row share the one scratch array; each equals bin_particles
    on the same request and the oracle.  Sizes: a partition-strategy request
    (1024^2 grid, ragged n, two attributes), then smaller ones - a whole-grid
    LDS request with bounds from the data and a small partition request."""
    big = (3_000_017, 1024, 2, 1, (0.0, 1.0, 0.0, 1.0))
    lds = (50_001, 64, 1, 2, None)
    small = (1_001, 1024, 1, 3, (0.0, 1.0, 0.0, 1.0))
    seq = [big, lds, small] if order == "large_then_small" else [lds, big, small]
    s_na = torch.cuda.Stream()
    s_pl = torch.cuda.Stream()
    for (n, side, k, seed, bounds) in seq:
        _case(f"noalloc n={n} side={side} k={k} bounds={'data' if bounds is None else 'given'}")
        ws = _ws(n, side, k, seed)
        got = _run(B.bin_particles_noalloc, ws, bounds, s_na)
        ref = _run(B.bin_particles, ws, bounds, s_pl)
        _same_as_plain_call(got, ref)
        ref_orc = orc.bin_particles(ws.coords, ws.attrs, ws.axes, bounds, ws.nx, ws.ny)
        G.assert_parity(got, ref_orc, B.OPS_ALL, what=f"noalloc n={n}")


def test_noalloc_takes_no_device_memory():
    """A call whose plan needs ~100 MB of scratch leaves the device's free
    memory unchanged (bin_particles would grow its pool by that much)."""
    _case("noalloc free memory")
    s = torch.cuda.Stream()
    warm = _ws(1000, 64, 1, 5)
    _run(B.bin_particles_noalloc, warm, warm.bounds, s)  # the array is resident from here on
    n = 12_000_000
    ws = _ws(n, 2048, 1, 6)
    coords, attrs = G.to_device(ws)
    out = B.alloc_outputs(attrs, ws.nx, ws.ny, B.OPS_ALL, "cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    B.bin_particles_noalloc(coords, attrs, n, ws.axes, ws.bounds, ws.nx, ws.ny, B.OPS_ALL, out, stream=s)
    s.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (16 << 20), (free0, free1)
    got = _to_np(out)
    assert int(got["count"].sum()) == int(np.sum((ws.coords[0] >= 0) & (ws.coords[0] <= 1)
                                                 & (ws.coords[1] >= 0) & (ws.coords[1] <= 1)))


def test_noalloc_refuses_requests_beyond_its_array():
    """64M particles on a 2048^2 grid need more scratch than the array holds:
    BIN_ERR_INVALID_ARG naming the limit, nothing enqueued (the outputs keep
    their fill), and the next call on the same stream works."""
    _case("noalloc too large")
    s = torch.cuda.Stream()
    n = 1 << 26
    coords = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(2)]
    attrs = [torch.ones(n, dtype=torch.float32, device="cuda")]
    out = B.alloc_outputs(attrs, 2048, 2048, B.OPS_ALL, "cuda")
    out["count"].fill_(7)
    torch.cuda.synchronize()
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_noalloc(coords, attrs, n, (0, 1), (0.0, 1.0, 0.0, 1.0), 2048, 2048, B.OPS_ALL, out,
                                stream=s)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    assert "allocation-free" in str(ei.value) and str(256 << 20) in str(ei.value)
    s.synchronize()
    assert bool((out["count"] == 7).all())
    small = _ws(4097, 32, 1, 9)
    got = _run(B.bin_particles_noalloc, small, small.bounds, s)
    G.assert_parity(got, G.oracle(small), B.OPS_ALL, what="after refusal")
