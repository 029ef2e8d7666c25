"""CPU oracle for in situ particle data binning.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may call
this module.  The product path (the HIP library and its binding) never
imports it and shares no code with it.

What is computed (paper, Section 4.2): the particle table has one column per
variable and one row per particle.  Two chosen variables are the axes of a
uniform Cartesian mesh whose axis bounds are given; the coordinate values of
a particle select the mesh cell ("bin") it belongs to.  Per bin, a counter is
incremented (a histogram), and every other requested variable is reduced by
sum, minimum, maximum and average.

The paper leaves the following points open.  The readings taken here (and by
the HIP path) are:

* R1 closed upper edge: a particle with ``x == hi`` belongs to the last bin;
  a particle is inside iff ``lo <= x <= hi`` on both axes.
* R2 index arithmetic, IEEE binary64 with round-to-nearest-even, no fused
  multiply-add: ``s = nbins / (hi - lo)`` once per axis, then
  ``i = trunc((x - lo) * s)``, clamped to ``nbins - 1``.  Coordinates are
  first widened exactly to binary64.
* R3 particles outside the bounds, or with a NaN/Inf coordinate, take part in
  no reduction.
* R4 empty bins: count 0, sum 0, min +Inf, max -Inf, avg NaN.
* R5 avg = sum / count, formed from the binary64 sum.
* R6 min and max follow IEEE 754 totalOrder on non-NaN values (so -0 < +0).
* R7 bins are cells, stored row-major ``[ny][nx]`` with flat index
  ``iy * nx + ix``; with one or three axes (``bin_particles_nd``) axis 0
  still varies fastest: ``[nz][ny][nx]``, flat ``(iz * ny + iy) * nx + ix``.
* R8 sums are reference values in binary64; besides them the oracle reports
  ``abs_sum`` = per-bin sum of |a|, the scale used by sum tolerances.
* R9 bounds taken from the data (``bounds=None``): per axis the minimum and
  maximum over the finite coordinate values; with the closed upper edge the
  extreme particles land in the first and last cell.  A zero-extent axis
  (all finite values equal) puts them all in its first cell, as does an
  axis whose extent ``hi - lo`` or scale ``nbins / (hi - lo)`` is not finite
  in binary64; an axis with no finite value leaves every bin empty.

Parity pins: brute force (exact rational index, exactly rounded sums) on
small inputs; SciPy ``binned_statistic_2d`` / ``binned_statistic`` /
``binned_statistic_dd`` and NumPy ``histogram2d`` / ``histogram`` /
``histogramdd``; hand-worked cases; marginals of 3-D meshes; invariants and
metamorphic relations.  See tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence

import numpy as np

COUNT, SUM, MIN, MAX, AVG = 1, 2, 4, 8, 16
ALL_OPS = COUNT | SUM | MIN | MAX | AVG

_I64_MAX_MAG = np.int64(0x7FFFFFFFFFFFFFFF)


def axis_index(v, lo: float, hi: float, nbins: int):
    """Inside-mask and bin index along one axis (Section 4.2; readings R1-R3).

    ``v`` is widened to binary64; ``lo``/``hi`` are binary64 bounds.
    Returns ``(inside, idx)``; ``idx`` is meaningful only where ``inside``.
    """
    v = np.asarray(v).astype(np.float64)
    lo = np.float64(lo)
    hi = np.float64(hi)
    with np.errstate(invalid="ignore"):
        inside = (v >= lo) & (v <= hi)
    # R9: an axis of zero extent (possible only with bounds taken from the
    # data) puts every inside particle into its first cell, and so does one
    # whose extent hi - lo or scale nbins / (hi - lo) is not finite in
    # binary64 (data spanning more than the largest double, or a subnormal
    # extent): R2 has no finite scale to multiply by.
    with np.errstate(over="ignore", divide="ignore"):
        scale = np.float64(nbins) / (hi - lo) if hi > lo else np.float64(0.0)
        if not (np.isfinite(hi - lo) and np.isfinite(scale)):
            scale = np.float64(0.0)
    idx = np.zeros(v.shape, dtype=np.int64)
    if scale > 0:
        t = (v[inside] - lo) * scale
        idx[inside] = np.trunc(t).astype(np.int64)
    np.minimum(idx, nbins - 1, out=idx)
    return inside, idx


def auto_bounds(coords: Sequence[np.ndarray], axes) -> tuple:
    """Mesh bounds taken from the data (Section 4.2: the minimum and maximum
    of each coordinate variable), over finite values only (reading R9).  An
    axis column without a finite value gives (+Inf, -Inf): nothing is inside."""
    out = []
    for ax in axes:
        v = np.asarray(coords[ax]).astype(np.float64)
        f = v[np.isfinite(v)]
        out += [float(f.min()), float(f.max())] if f.size else [np.inf, -np.inf]
    return tuple(out)


def flat_bins(coords: Sequence[np.ndarray], axes, bounds, nx: int, ny: int):
    """Flat bin index of every particle inside the mesh, and the inside mask (R7)."""
    inx, ix = axis_index(coords[axes[0]], bounds[0], bounds[1], nx)
    iny, iy = axis_index(coords[axes[1]], bounds[2], bounds[3], ny)
    inside = inx & iny
    return inside, (iy * nx + ix)[inside]


def total_order_key(a: np.ndarray) -> np.ndarray:
    """Integer keys whose signed order is IEEE totalOrder of binary64 (R6)."""
    bits = np.ascontiguousarray(a, dtype=np.float64).view(np.int64)
    return np.where(bits >= 0, bits, bits ^ _I64_MAX_MAG)


def from_total_order_key(k: np.ndarray) -> np.ndarray:
    bits = np.where(k >= 0, k, k ^ _I64_MAX_MAG)
    return bits.astype(np.int64).view(np.float64)


def bin_particles(coords: Sequence[np.ndarray], attrs: Sequence[np.ndarray], axes=(0, 1),
                  bounds=(0.0, 1.0, 0.0, 1.0), nx: int = 64, ny: int = 64,
                  ops: int = ALL_OPS) -> Dict[str, object]:
    """Bin particles onto an ``ny`` x ``nx`` mesh and reduce per bin, in binary64.

    Returns a dict with ``count`` (int64, [ny, nx]), and per attribute lists
    ``sum``, ``min``, ``max``, ``avg``, ``abs_sum`` (float64, [ny, nx]).
    Every op is computed; ``ops`` is accepted for signature symmetry only.
    Also ``inside`` = the number of particles inside the mesh.
    """
    if bounds is None:
        bounds = auto_bounds(coords, axes)
    inside, b = flat_bins(coords, axes, bounds, nx, ny)
    return _reduce_bins(inside, b, attrs, (ny, nx))


def bin_particles_nd(coords: Sequence[np.ndarray], attrs: Sequence[np.ndarray], axes=(0, 1, 2),
                     bounds=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0), dims=(16, 16, 16),
                     ops: int = ALL_OPS) -> Dict[str, object]:
    """Bin onto a mesh of one, two or three axes (Section 4.2: the mesh axes
    are any chosen subset of the particle variables).

    ``axes[j]`` names the column of axis j, ``bounds[2j], bounds[2j+1]`` its
    lower and upper bound, ``dims[j]`` its number of bins.  Every axis follows
    R1-R3 on its own; a particle is inside iff it is inside on every axis.
    Row-major generalised from R7: axis 0 varies fastest, so the result arrays
    have shape ``dims`` reversed and the flat index is
    ``i0 + dims[0] * (i1 + dims[1] * i2)``.  ``bounds=None`` takes every axis's
    bounds from the data (R9).
    """
    d = len(axes)
    if not 1 <= d <= 3 or len(dims) != d:
        raise ValueError("one to three axes, one bin count per axis")
    if bounds is None:
        bounds = auto_bounds(coords, axes)
    n = len(coords[axes[0]])
    inside = np.ones(n, dtype=bool)
    flat = np.zeros(n, dtype=np.int64)
    stride = 1
    for j in range(d):
        inj, ij = axis_index(coords[axes[j]], bounds[2 * j], bounds[2 * j + 1], dims[j])
        inside &= inj
        flat += ij * stride
        stride *= int(dims[j])
    return _reduce_bins(inside, flat[inside], attrs, tuple(int(v) for v in reversed(dims)))


def _reduce_bins(inside, b, attrs, shape) -> Dict[str, object]:
    """Per-bin count, and per attribute sum/min/max/avg/abs_sum (R4-R6, R8),
    of the inside particles whose flat bin indices are ``b``."""
    nb = int(np.prod(shape))
    count = np.bincount(b, minlength=nb).astype(np.int64)
    res = {"count": count.reshape(shape), "sum": [], "min": [], "max": [], "avg": [],
           "abs_sum": [], "inside": int(inside.sum())}
    empty = count == 0
    for a in attrs:
        a64 = np.asarray(a).astype(np.float64)[inside]
        s = np.bincount(b, weights=a64, minlength=nb)
        asum = np.bincount(b, weights=np.abs(a64), minlength=nb)
        keys = total_order_key(a64)
        kmin = np.full(nb, total_order_key(np.array([np.inf]))[0], dtype=np.int64)
        kmax = np.full(nb, total_order_key(np.array([-np.inf]))[0], dtype=np.int64)
        np.minimum.at(kmin, b, keys)
        np.maximum.at(kmax, b, keys)
        mn = from_total_order_key(kmin)
        mx = from_total_order_key(kmax)
        with np.errstate(invalid="ignore", divide="ignore"):
            avg = np.where(empty, np.nan, s / np.maximum(count, 1))
        s = np.where(empty, 0.0, s)
        res["sum"].append(s.reshape(shape))
        res["min"].append(mn.reshape(shape))
        res["max"].append(mx.reshape(shape))
        res["avg"].append(avg.reshape(shape))
        res["abs_sum"].append(asum.reshape(shape))
    return res


def merge(parts: List[Dict[str, object]]) -> Dict[str, object]:
    """Combine results of disjoint particle sets (counts and sums add, min of
    mins, max of maxes, avg re-formed).  Used to state the merge law in tests
    and to split the CPU baseline over processes."""
    out = {"count": sum(p["count"] for p in parts), "inside": sum(p["inside"] for p in parts),
           "sum": [], "min": [], "max": [], "avg": [], "abs_sum": []}
    k = len(parts[0]["sum"])
    empty = out["count"] == 0
    for j in range(k):
        s = sum(p["sum"][j] for p in parts)
        out["sum"].append(s)
        out["abs_sum"].append(sum(p["abs_sum"][j] for p in parts))
        kmin = np.minimum.reduce([total_order_key(p["min"][j].ravel()) for p in parts])
        kmax = np.maximum.reduce([total_order_key(p["max"][j].ravel()) for p in parts])
        out["min"].append(from_total_order_key(kmin).reshape(s.shape))
        out["max"].append(from_total_order_key(kmax).reshape(s.shape))
        with np.errstate(invalid="ignore", divide="ignore"):
            out["avg"].append(np.where(empty, np.nan, s / np.maximum(out["count"], 1)))
    return out


# --------------------------------------------------------------------------
# Brute force, for tiny inputs: exact rational arithmetic, no NumPy reductions.
# --------------------------------------------------------------------------

def _exact_index(v: float, lo: float, hi: float, nbins: int) -> Optional[int]:
    """Bin of ``v`` in exact rational arithmetic: floor((v-lo) * n / (hi-lo)),
    the last bin for ``v == hi``, None outside (R1, R3)."""
    if not (lo <= v <= hi):          # NaN compares false
        return None
    if lo == hi or not math.isfinite(hi - lo) or not math.isfinite(nbins / (hi - lo)):
        return 0                     # zero or unrepresentable extent (R9)
    i = math.floor((Fraction(v) - Fraction(lo)) * nbins / (Fraction(hi) - Fraction(lo)))
    return min(i, nbins - 1)


def _total_order_sort_key(v: float):
    # totalOrder on non-NaN values: numeric order, then -0 before +0.
    return (v, math.copysign(1.0, v))


def bin_particles_bruteforce(coords, attrs, axes=(0, 1), bounds=(0.0, 1.0, 0.0, 1.0),
                             nx: int = 4, ny: int = 4) -> Dict[str, object]:
    """Per-particle loop with the exact rational bin index and exactly rounded
    (``math.fsum``) per-bin sums.  Same result layout as ``bin_particles``."""
    n = len(coords[0])
    if bounds is None:               # R9, by plain Python min/max
        bl = []
        for ax in axes:
            vals = [float(v) for v in coords[ax] if math.isfinite(float(v))]
            bl += [min(vals), max(vals)] if vals else [math.inf, -math.inf]
        bounds = tuple(bl)
    members: List[List[int]] = [[] for _ in range(nx * ny)]
    for i in range(n):
        ix = _exact_index(float(coords[axes[0]][i]), bounds[0], bounds[1], nx)
        iy = _exact_index(float(coords[axes[1]][i]), bounds[2], bounds[3], ny)
        if ix is None or iy is None:
            continue
        members[iy * nx + ix].append(i)
    count = np.array([len(m) for m in members], dtype=np.int64).reshape(ny, nx)
    res = {"count": count, "sum": [], "min": [], "max": [], "avg": [], "abs_sum": [],
           "inside": int(count.sum())}
    for a in attrs:
        vals = [[float(a[i]) for i in m] for m in members]
        s = np.array([math.fsum(v) for v in vals]).reshape(ny, nx)
        asum = np.array([math.fsum(abs(x) for x in v) for v in vals]).reshape(ny, nx)
        mn = np.array([min(v, key=_total_order_sort_key) if v else math.inf for v in vals])
        mx = np.array([max(v, key=_total_order_sort_key) if v else -math.inf for v in vals])
        avg = np.array([float(Fraction(math.fsum(v)) / len(v)) if v else math.nan for v in vals])
        res["sum"].append(s)
        res["min"].append(mn.reshape(ny, nx))
        res["max"].append(mx.reshape(ny, nx))
        res["avg"].append(avg.reshape(ny, nx))
        res["abs_sum"].append(asum)
    return res


def bin_particles_nd_bruteforce(coords, attrs, axes, bounds, dims) -> Dict[str, object]:
    """Brute force for one to three axes: the exact rational bin on every
    axis, particles collected per cell tuple, cells laid out by NumPy's own
    C order over the shape ``dims`` reversed (so no flat-index arithmetic of
    its own), exactly rounded per-bin sums."""
    d = len(axes)
    if bounds is None:
        bl = []
        for ax in axes:
            vals = [float(v) for v in coords[ax] if math.isfinite(float(v))]
            bl += [min(vals), max(vals)] if vals else [math.inf, -math.inf]
        bounds = tuple(bl)
    shape = tuple(int(v) for v in reversed(dims))
    members: Dict[tuple, List[int]] = {cell: [] for cell in np.ndindex(*shape)}
    for i in range(len(coords[axes[0]])):
        idx = [_exact_index(float(coords[axes[j]][i]), bounds[2 * j], bounds[2 * j + 1], dims[j])
               for j in range(d)]
        if any(v is None for v in idx):
            continue
        members[tuple(reversed(idx))].append(i)
    count = np.zeros(shape, dtype=np.int64)
    for cell, m in members.items():
        count[cell] = len(m)
    res = {"count": count, "sum": [], "min": [], "max": [], "avg": [], "abs_sum": [],
           "inside": int(count.sum())}
    for a in attrs:
        s, asum, mn, mx, avg = (np.zeros(shape) for _ in range(5))
        for cell, m in members.items():
            v = [float(a[i]) for i in m]
            s[cell] = math.fsum(v)
            asum[cell] = math.fsum(abs(x) for x in v)
            mn[cell] = min(v, key=_total_order_sort_key) if v else math.inf
            mx[cell] = max(v, key=_total_order_sort_key) if v else -math.inf
            avg[cell] = float(Fraction(math.fsum(v)) / len(v)) if v else math.nan
        for key, arr in (("sum", s), ("min", mn), ("max", mx), ("avg", avg), ("abs_sum", asum)):
            res[key].append(arr)
    return res
