"""GPU results at the largest sizes the boundary accepts, checked bin by bin
against the closed forms of tests/lattice_pattern.py (pinned to the oracle
on the CPU).

- Particle counts up to 2^32 - 1, past every 32-bit signed index, with the
  automatic plan and the strategy it takes asserted: the tile partition with
  the quad gather (the largest n whose padded tile totals fit 32 bits), the
  partition with the record gather (at n = 2^32 - 1, and with four
  attributes), the whole grid in LDS; bounds given and from the data.
- Grids of 2^30 and 2^31 - 1 bins (global atomics).
- n = 2^32 - 1 on a three-axis mesh, in one batched call, and in the
  asynchronous mode."""
import sys

import numpy as np
import pytest

from tests import gpu_check as G
from tests import lattice_pattern as L

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
torch = pytest.importorskip("torch")

CHUNK = 1 << 27


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _fill(n, nx, ny, k):
    """The lattice columns built on the device, CHUNK particles at a time."""
    dev = torch.device("cuda:0")
    x = torch.empty(n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    attrs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(k)]
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        idx = torch.arange(s, e, dtype=torch.int64, device=dev)
        cx, cy, ca = L.columns(idx, nx, ny, k, lambda v: v.to(torch.float32))
        x[s:e] = cx
        y[s:e] = cy
        for j in range(k):
            attrs[j][s:e] = ca[j]
        del idx, cx, cy, ca
    torch.cuda.synchronize()
    return [x, y], attrs


@pytest.mark.parametrize("n,side,k,kind,quads,auto", [
    pytest.param((1 << 32) - (1 << 21) + 1, 2048, 1, "partition", "1", False, id="partition-quads-n=2^32-2^21+1"),
    pytest.param(0xFFFFFFFF, 2048, 1, "partition", "0", False, id="partition-records-n=2^32-1"),
    pytest.param((1 << 31) + 4097, 1024, 4, "partition", "0", False, id="partition-records-k4-n=2^31+4097"),
    pytest.param(0xFFFFFFFF, 64, 1, "lds", None, False, id="lds-n=2^32-1"),
    pytest.param((1 << 32) - (1 << 21) + 1, 2048, 1, "partition", "1", True, id="partition-quads-auto-bounds"),
    pytest.param(0xFFFFFFFF, 64, 1, "lds", None, True, id="lds-auto-bounds-n=2^32-1"),
])
def test_largest_particle_counts(n, side, k, kind, quads, auto):
    """auto: bounds from the data (every cell centre occurs, so the closed
    form still holds)."""
    from paper_2310_02926_amd import binding as B
    need = n * (10 + 8 * k) + (8 << 30)  # columns, records (2-byte bin, values) and slack
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    _case(f"largest counts n={n} grid={side}^2 k={k} auto bounds={auto} expected plan={kind}")
    B.bin_set_plan_override(-1, 0, 0)
    coords, attrs = _fill(n, side, side, k)
    out = B.alloc_outputs(attrs, side, side, B.OPS_ALL, torch.device("cuda:0"))
    bounds = (0.0, 1.0, 0.0, 1.0)
    req, keep = B.request(coords, attrs, n, (0, 1), bounds, side, side, B.OPS_ALL,
                          {key: (v.view(-1) if not isinstance(v, list) else [t.view(-1) for t in v])
                           for key, v in out.items()})
    plan = B.bin_describe_plan(req)
    _case(f"plan: {plan}")
    assert plan.split()[0] == kind
    if quads is not None:
        assert f"quads={quads}" in plan
    stream = torch.cuda.Stream()
    try:
        B.bin_particles(coords, attrs, n, (0, 1), None if auto else bounds, side, side, B.OPS_ALL, out,
                        stream=stream)
        stream.synchronize()
        got = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
        for key in ("sum", "min", "max", "avg"):
            got[key] = [t.cpu().numpy() for t in out[key]]
    finally:
        del coords, attrs, out, req, keep
        torch.cuda.synchronize()
        B.bin_release_workspace()
        torch.cuda.empty_cache()
    exp = L.expected(n, side, side, k)
    assert int(got["count"].sum()) == n
    G.assert_parity(got, exp, B.OPS_ALL, what=f"n={n} {side}^2 k={k}")


@pytest.mark.parametrize("n,nx,ny,f64", L.MAX_GRID_CASES, ids=L.MAX_GRID_IDS)
def test_largest_grids(n, nx, ny, f64):
    """Grids of 2^30 and 2^31 - 1 bins (global atomics), the sparse pattern
    reaching the last row: every used bin holds its one particle, every
    other bin the empty-bin values.  Checked on the device (the outputs are
    tens of GB)."""
    from paper_2310_02926_amd import binding as B
    nb = nx * ny
    need = nb * 28 + n * 24 + (8 << 30)  # outputs, columns and slack
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    _case(f"largest grids n={n} grid={nx}x{ny} f64 coords={f64}")
    B.bin_set_plan_override(-1, 0, 0)
    dev = torch.device("cuda:0")
    ct = torch.float64 if f64 else torch.float32
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    x, y, attrs = L.sparse_columns(idx, n, nx, ny, 1, lambda v: v.to(ct))
    attrs = [a.to(torch.float32) for a in attrs]
    out = B.alloc_outputs(attrs, nx, ny, B.OPS_ALL, dev)
    bounds = (0.0, 1.0, 0.0, 1.0)
    req, keep = B.request([x, y], attrs, n, (0, 1), bounds, nx, ny, B.OPS_ALL,
                          {key: (v.view(-1) if not isinstance(v, list) else [t.view(-1) for t in v])
                           for key, v in out.items()})
    plan = B.bin_describe_plan(req)
    _case(f"plan: {plan}")
    assert plan.split()[0] == "global"
    stream = torch.cuda.Stream()
    try:
        B.bin_particles([x, y], attrs, n, (0, 1), bounds, nx, ny, B.OPS_ALL, out, stream=stream)
        stream.synchronize()
        cells = L.sparse_cells(idx, n, nx, ny)
        v = attrs[0]
        cnt = out["count"].view(-1)
        assert int(torch.count_nonzero(cnt)) == n
        assert bool((cnt[cells] == 1).all())
        s, mn, mx, av = (out[key][0].view(-1) for key in ("sum", "min", "max", "avg"))
        assert bool((s[cells] == v.to(s.dtype)).all())
        assert int(torch.count_nonzero(s)) == int(torch.count_nonzero(v))
        assert bool((mn[cells] == v).all()) and bool((mx[cells] == v).all())
        assert int((mn == float("inf")).sum()) == nb - n
        assert int((mx == float("-inf")).sum()) == nb - n
        assert bool((av[cells] == v.to(av.dtype)).all())
        assert int(torch.isnan(av).sum()) == nb - n
    finally:
        del x, y, attrs, out, req, keep, idx
        torch.cuda.synchronize()
        B.bin_release_workspace()
        torch.cuda.empty_cache()


def test_largest_particle_count_three_axes():
    """n = 2^32 - 1 on a 64^3 mesh: the fold's composite column and the
    folded two-axis binning at the largest n, against the closed form."""
    from paper_2310_02926_amd import binding as B
    n, d = 0xFFFFFFFF, 64
    need = n * 26 + (8 << 30)  # four columns, the composite column, records, slack
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    _case(f"largest count, three axes: n={n} mesh={d}^3")
    B.bin_set_plan_override(-1, 0, 0)
    dev = torch.device("cuda:0")
    cols = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4)]
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        idx = torch.arange(s, e, dtype=torch.int64, device=dev)
        x, y, z, attrs = L.columns3(idx, d, d, d, 1, lambda v: v.to(torch.float32))
        for c, v in zip(cols, (x, y, z, attrs[0])):
            c[s:e] = v
        del idx, x, y, z, attrs
    torch.cuda.synchronize()
    dims = (d, d, d)
    out = B.alloc_outputs_nd(cols[3:], dims, B.OPS_ALL, dev)
    stream = torch.cuda.Stream()
    try:
        B.bin_particles_nd(cols[:3], cols[3:], n, (0, 1, 2), (0.0, 1.0) * 3, dims, B.OPS_ALL, out, stream=stream)
        stream.synchronize()
        got = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
        for key in ("sum", "min", "max", "avg"):
            got[key] = [t.cpu().numpy() for t in out[key]]
    finally:
        del cols, out
        torch.cuda.synchronize()
        B.bin_release_workspace()
        torch.cuda.empty_cache()
    exp = L.expected3(n, d, d, d, 1)
    assert got["count"].shape == (d, d, d)
    assert int(got["count"].sum()) == n
    G.assert_parity(got, exp, B.OPS_ALL, what=f"three axes n={n} {d}^3")


def test_largest_particle_counts_in_one_batch():
    """One batched call holding a partition request at n = 2^31 + 4097
    (1024^2), a whole-grid-in-LDS request at n = 2^32 - 1 (64^2) and a small
    ragged one with two attributes (256^2): each against its closed form."""
    from paper_2310_02926_amd import binding as B
    cases = [((1 << 31) + 4097, 1024, 1), (0xFFFFFFFF, 64, 1), (100_003, 256, 2)]
    need = sum(n * (12 + 4 * k) for n, _, k in cases) + (8 << 30)  # columns, records, slack
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    _case(f"largest counts in one batch: {cases}")
    B.bin_set_plan_override(-1, 0, 0)
    dev = torch.device("cuda:0")
    reqs = []
    for n, side, k in cases:
        coords, attrs = _fill(n, side, side, k)
        out = B.alloc_outputs(attrs, side, side, B.OPS_ALL, dev)
        reqs.append(dict(coords=coords, attrs=attrs, n=n, axes=(0, 1), bounds=(0.0, 1.0, 0.0, 1.0), nx=side,
                         ny=side, ops=B.OPS_ALL, out=out))
    stream = torch.cuda.Stream()
    gots = []
    try:
        B.bin_particles_batched(reqs, stream=stream)
        stream.synchronize()
        for r in reqs:
            got = {"count": r["out"]["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
            for key in ("sum", "min", "max", "avg"):
                got[key] = [t.cpu().numpy() for t in r["out"][key]]
            gots.append(got)
    finally:
        del reqs
        torch.cuda.synchronize()
        B.bin_release_workspace()
        torch.cuda.empty_cache()
    for (n, side, k), got in zip(cases, gots):
        assert int(got["count"].sum()) == n
        G.assert_parity(got, L.expected(n, side, side, k), B.OPS_ALL, what=f"batched n={n} {side}^2 k={k}")


def test_largest_particle_count_async():
    """The asynchronous in situ mode at n = 2^32 - 1 (64^2): the deep copy
    is taken in the source stream's order, the source columns are then
    overwritten on that stream, and the grids still hold the lattice's
    closed form."""
    from paper_2310_02926_amd import binding as B
    n, side = 0xFFFFFFFF, 64
    need = n * 24 + (8 << 30)  # columns and their staged copy, slack
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    _case(f"largest count, asynchronous mode: n={n} grid={side}^2")
    B.bin_set_plan_override(-1, 0, 0)
    coords, attrs = _fill(n, side, side, 1)
    out = B.alloc_outputs(attrs, side, side, B.OPS_ALL, torch.device("cuda:0"))
    src, bs = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        with torch.cuda.stream(src):
            B.bin_particles_async(coords, attrs, n, (0, 1), (0.0, 1.0, 0.0, 1.0), side, side, B.OPS_ALL, out,
                                  src_stream=src, bin_stream=bs)
            coords[0].fill_(2.0)  # after the copy in src's order: every particle outside
            attrs[0].fill_(5.0)
        torch.cuda.synchronize()
        got = {"count": out["count"].cpu().numpy().view(np.uint32).astype(np.int64)}
        for key in ("sum", "min", "max", "avg"):
            got[key] = [t.cpu().numpy() for t in out[key]]
    finally:
        del coords, attrs, out
        torch.cuda.synchronize()
        B.bin_release_workspace()
        torch.cuda.empty_cache()
    assert int(got["count"].sum()) == n
    G.assert_parity(got, L.expected(n, side, side, 1), B.OPS_ALL, what=f"async n={n} {side}^2")
