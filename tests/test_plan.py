"""The planner's decisions without a GPU (bin_describe_plan_on): strategy,
tile size, gather kind, launch shape and the work-item bound, for the
device sizes of MI355X and of smaller parts."""
import re

import numpy as np
from ctypes import c_double, c_int32

import pytest

from paper_2310_02926_amd import binding as B

F = 0x10000  # fake, aligned device addresses: never dereferenced


def _req(n, nx, ny, k=1, f64c=False, f64a=False, ops=31, shift=0):
    coords = [F + shift * (8 if f64c else 4), F + 0x100]
    attrs = [F + 0x200 + 0x100 * j for j in range(k)]
    c, ck = B.columns(coords, B.BIN_F64 if f64c else B.BIN_F32)
    a, ak = B.columns(attrs, B.BIN_F64 if f64a else B.BIN_F32) if k else (B.Columns(None, 0, B.BIN_F32), None)
    lists = [[F + 0x2000 + 0x100 * j for j in range(k)] if (k and ops & bit) else None for bit in (2, 4, 8, 16)]
    o, ok = B.output(F + 0x1000 if ops & 1 else None, *lists)
    r = B.Request(c, a, n, (c_int32 * 2)(0, 1), (c_double * 4)(0.0, 1.0, 0.0, 1.0), nx, ny, ops, o)
    return r, (ck, ak, ok)


def plan(n, nx, ny, k=1, cus=256, lds=163840, **kw):
    r, keep = _req(n, nx, ny, k, **kw)
    text = B.bin_describe_plan_on(r, cus, lds, lds)
    fields = dict(re.findall(r"(\w+)=(\S+)", text))
    return text.split()[0], fields


def test_headline_plan():
    """2^27 particles on 2048^2 with one f32 attribute: 512 tiles of 8192
    bins (a tile's count, binary64 sum, min and max fill the 160 KB of
    LDS), 1024-thread scatter of 16 particles per thread, quad gather."""
    kind, f = plan(1 << 27, 2048, 2048)
    assert kind == "partition"
    assert f["tiles"] == "512" and f["tile_bins"] == "8192"
    assert f["threads"] == "1024" and f["ppt"] == "16" and f["quads"] == "1"
    assert int(f["bin_lds"]) == 8192 * 20 and f["vec"] == "1" and f["prec"] == "fp64"


def test_four_attributes_gather_record_by_record():
    kind, f = plan(1 << 24, 1024, 1024, k=4)
    assert kind == "partition" and f["quads"] == "0" and f["tile_bins"] == "2048"
    assert int(f["ppt"]) <= 8  # multi-attribute sub-chunks hold at most 8192 particles


def test_quads_only_for_one_f32_attribute_and_long_runs():
    assert plan(1 << 24, 2048, 2048, k=0, ops=1)[1]["quads"] == "1"
    assert plan(1 << 24, 2048, 2048, k=1, f64a=True)[1]["quads"] == "0"
    assert plan(1 << 24, 2048, 2048, k=2)[1]["quads"] == "0"
    # 4096 tiles of a 4096^2 grid: sub-chunks average < 16 records per tile
    assert plan(1 << 24, 4096, 4096, k=1)[1]["quads"] == "0"


def test_tiles_not_below_256_bins():
    """Small grids shrink tiles towards two per CU, but not below 256 bins."""
    for side in (128, 181, 256, 300):
        kind, f = plan(1 << 24, side, side)
        assert kind == "partition", side
        assert int(f["tile_bins"]) >= 256, (side, f)
    assert plan(1 << 24, 512, 512)[1]["tile_bins"] == "512"  # 512 tiles: two per CU
    # a smaller device keeps larger tiles
    assert int(plan(1 << 24, 512, 512, cus=64)[1]["tile_bins"]) > 512


def test_quads_only_while_padded_tile_totals_fit_32_bits():
    """A tile's record total, with up to 3 padding records per sub-chunk, is
    a 32-bit count: at the largest n the record gather is taken."""
    kind, f = plan(0xFFFFFFFF, 2048, 2048)
    assert kind == "partition" and f["quads"] == "0"
    rows = int(f["wg"]) * int(f["blocks"])
    n = 0xFFFFFFFF - 3 * rows
    assert plan(n, 2048, 2048)[1]["quads"] == "1"
    assert plan(n + 1, 2048, 2048)[1]["quads"] == "0"


def test_lds_strategy_at_most_1024_threads_per_cu():
    kind, f = plan(1 << 24, 64, 64)
    assert kind == "lds" and f["block"] == "1024" and f["grid"] == "256"
    kind, f = plan(1 << 24, 32, 32)
    assert kind == "lds" and f["block"] == "512" and f["grid"] == "512"
    kind, f = plan(1 << 24, 32, 32, cus=80)
    assert f["grid"] == "160"
    # few particles: fewer workgroups, each with at least 2 * bins particles
    kind, f = plan(65536, 64, 64)
    assert kind == "lds" and int(f["grid"]) <= 4


def test_work_item_bound_covers_padding():
    """max_items = tiles + floor(record slots / split_len), with the record
    slots including the quad padding of every sub-chunk."""
    for n, side, k in [(1 << 27, 2048, 1), (1 << 24, 1024, 4), (3_000_001, 700, 1), (1 << 24, 128, 1)]:
        kind, f = plan(n, side, side, k=k)
        assert kind == "partition"
        tiles, split, items = int(f["tiles"]), int(f["split"]), int(f["max_items"])
        nrows = int(f["wg"]) * int(f["blocks"])
        pad = 0
        if f["quads"] == "1":
            pad = (3 * min(tiles, int(f["sub"])) + 3) // 4 * 4
        slots = n + nrows * pad + 4
        assert items == tiles + slots // split, (n, side, f)


def _walk_items(counts, split_len):
    """The work-item rule of the tile binning, written out per tile: slice w
    opens item floor(excl(w) / split_len) of its tile, where excl(w) is the
    tile's records in earlier slices; an item starts at every slice whose
    number differs from the previous slice's.  Returns items per tile."""
    out = []
    for row in counts:
        excl, prev, items = 0, None, 0
        for c in row:
            m = excl // split_len
            if m != prev:
                items += 1
                prev = m
            excl += int(c)
        out.append(items)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_work_item_and_slot_bounds_hold_for_any_counts(seed):
    """The planner's bounds - items <= tiles + floor(R / L) and partial
    slots (items of tiles with two or more items) <= 2 floor(R / L) for R
    records in all - hold for every count matrix: random, one heavy slice,
    records just above multiples of L, all records in one tile."""
    rng = np.random.default_rng(seed)
    tiles, slices = int(rng.integers(1, 40)), int(rng.integers(1, 60))
    L = int(rng.integers(1, 50))
    kind = seed % 4
    if kind == 0:
        counts = rng.integers(0, 3 * L, (tiles, slices))
    elif kind == 1:
        counts = np.zeros((tiles, slices), dtype=np.int64)
        counts[:, rng.integers(0, slices)] = rng.integers(0, 20 * L, tiles)
    elif kind == 2:
        counts = np.full((tiles, slices), L + 1)
        counts[:, ::3] = 0
    else:
        counts = np.zeros((tiles, slices), dtype=np.int64)
        counts[rng.integers(0, tiles)] = rng.integers(L - 1, L + 2, slices)
    R = int(counts.sum())
    items = _walk_items(counts, L)
    assert sum(items) <= tiles + R // L
    assert sum(i for i in items if i > 1) <= 2 * (R // L)


def test_unaligned_columns_turn_off_wide_loads():
    assert plan(1 << 24, 2048, 2048, shift=1)[1]["vec"] == "0"
    assert plan(1 << 24, 2048, 2048, shift=0)[1]["vec"] == "1"


def test_large_grids_fall_back_to_global_atomics():
    # more than 4096 tiles of the largest LDS tile
    kind, f = plan(1 << 20, 16384, 8192, k=4)
    assert kind == "global"


@pytest.mark.parametrize("cus,lds_block,lds_cu", [(0, 163840, 163840), (256, 512, 163840), (256, 163840, 65536)])
def test_describe_plan_on_rejects_bad_device(cus, lds_block, lds_cu):
    r, keep = _req(1000, 64, 64)
    buf = __import__("ctypes").create_string_buffer(256)
    st = B.lib().bin_describe_plan_on(__import__("ctypes").byref(r), cus, lds_block, lds_cu, buf, 256)
    assert st == B.BIN_ERR_INVALID_ARG
