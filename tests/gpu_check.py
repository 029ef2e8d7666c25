"""Helpers for GPU parity tests: run the HIP path through the C ABI on a
workload and compare with the CPU oracle element by element."""
from __future__ import annotations

import numpy as np

from oracle import binning_oracle as orc

# Sum/avg tolerance: |got - ref| <= REL * sum|a| per bin (relative error for
# non-negative attributes).  Holds for the compensated FP32 and the FP64
# accumulation paths; the plain FP32 path is checked against a bound that
# grows with the bin's count instead (see plain_bound).
REL = 1e-5
# Besides the sum|a|-normalised bound, the compensated and binary64 paths are
# held to plain relative error against the FP64 reference on every bin whose
# sum is not cancelled: |ref| >= sum|a| / COND_MAX (condition number at most
# COND_MAX).  Where a signed attribute's sum cancels, relative error is not
# defined by the data and only the normalised bound applies.
COND_MAX = 1e3


def to_device(ws, device="cuda"):
    import torch
    coords = [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in ws.coords]
    attrs = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in ws.attrs]
    return coords, attrs


def run_gpu(ws, ops=None, axes=None, bounds=None, stream=None, coords=None, attrs=None):
    """Bin a synth.Workload on the GPU; returns numpy results shaped [ny, nx]."""
    import torch
    from paper_2310_02926_amd import binding as B
    if coords is None:
        coords, attrs = to_device(ws)
    ops = ws.ops if ops is None else ops
    out = B.bin_particles_alloc(coords, attrs, axes or ws.axes, ws.bounds if bounds is None else bounds,
                                ws.nx, ws.ny, ops, stream=stream)
    torch.cuda.synchronize()
    res = {}
    if "count" in out:
        res["count"] = out["count"].cpu().numpy().view(np.uint32).astype(np.int64)
    for key in ("sum", "min", "max", "avg"):
        if key in out:
            res[key] = [t.cpu().numpy() for t in out[key]]
    return res


def assert_parity(got, ref, ops, rel=REL, plain=False, what=""):
    """count/min/max bit-exact; sum/avg within tolerance; empty-bin values."""
    from paper_2310_02926_amd import binding as B
    cnt = ref["count"]
    empty = cnt == 0
    if ops & B.COUNT:
        assert np.array_equal(got["count"], cnt), f"{what}: count differs in {np.sum(got['count'] != cnt)} bins"
    k = len(ref["sum"])
    for j in range(k):
        if ops & B.MIN:
            g = got["min"][j]
            r = ref["min"][j].astype(g.dtype)
            bad = g.view(np.int64 if g.dtype == np.float64 else np.int32) != r.view(
                np.int64 if g.dtype == np.float64 else np.int32)
            assert not bad.any(), f"{what}: min[{j}] differs in {bad.sum()} bins, e.g. {np.argwhere(bad)[:3]}"
        if ops & B.MAX:
            g = got["max"][j]
            r = ref["max"][j].astype(g.dtype)
            bad = g.view(np.int64 if g.dtype == np.float64 else np.int32) != r.view(
                np.int64 if g.dtype == np.float64 else np.int32)
            assert not bad.any(), f"{what}: max[{j}] differs in {bad.sum()} bins"
        bound = ref["abs_sum"][j] * (plain_bound(cnt) if plain else rel)
        if ops & B.SUM:
            g = got["sum"][j].astype(np.float64)
            err = np.abs(g - ref["sum"][j])
            bad = ~(err <= bound)
            assert not bad.any(), (f"{what}: sum[{j}] off in {bad.sum()} bins; worst excess "
                                   f"{np.max((err - bound)[bad])}")
            assert np.all(g[empty] == 0), f"{what}: empty-bin sum not 0"
            if not plain:
                r = ref["sum"][j]
                well = ~empty & (np.abs(r) * COND_MAX >= ref["abs_sum"][j])
                rbad = well & ~(err <= rel * np.abs(r))
                assert not rbad.any(), (f"{what}: sum[{j}] relative error above {rel} in {rbad.sum()} "
                                        f"well-conditioned bins")
        if ops & B.AVG:
            g = got["avg"][j].astype(np.float64)
            err = np.abs(g - ref["avg"][j])
            with np.errstate(invalid="ignore", divide="ignore"):
                ok = err <= bound / np.maximum(cnt, 1) + _avg_cast_slack(got["avg"][j].dtype, ref["avg"][j])
            ok = np.where(empty, np.isnan(g), ok)
            assert ok.all(), f"{what}: avg[{j}] off in {np.sum(~ok)} bins"
            if not plain:
                r = ref["avg"][j]
                with np.errstate(invalid="ignore"):
                    well = ~empty & (np.abs(r) * cnt * COND_MAX >= ref["abs_sum"][j])
                    slack = _avg_cast_slack(got["avg"][j].dtype, r)
                    rbad = well & ~(err <= rel * np.abs(r) + slack)
                assert not rbad.any(), (f"{what}: avg[{j}] relative error above {rel} in {rbad.sum()} "
                                        f"well-conditioned bins")


def _avg_cast_slack(dtype, ref_avg):
    # A float32 avg output carries its own rounding (half an ulp).
    if dtype == np.float32:
        with np.errstate(invalid="ignore"):
            return np.nan_to_num(np.abs(ref_avg) * 2.0 ** -24)
    return 0.0


def plain_bound(count):
    """Error bound of a sequential FP32 sum of c terms plus the final float
    rounding: (c + 1) * 2^-24 * sum|a| (relative to sum|a|)."""
    return (count + 1) * 2.0 ** -24


def oracle(ws, axes=None, bounds=None):
    return orc.bin_particles(ws.coords, ws.attrs, axes or ws.axes, ws.bounds if bounds is None else bounds,
                             ws.nx, ws.ny)
