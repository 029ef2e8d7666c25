"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pin suite catches every one of them.  This is what makes the pins
worth trusting: a pin that no mistake can fail pins nothing."""
import os
import types

import pytest

from tests import oracle_pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "binning_oracle.py")

# (name, text in the oracle, replacement).  Each text must occur exactly once.
MUTANTS = [
    ("open_upper_edge", "inside = (v >= lo) & (v <= hi)", "inside = (v >= lo) & (v < hi)"),
    ("nan_inside", "inside = (v >= lo) & (v <= hi)", "inside = ~((v < lo) | (v > hi))"),
    ("no_clamp", "np.minimum(idx, nbins - 1, out=idx)", "pass"),
    ("ceil_not_trunc", "np.trunc(t)", "np.ceil(t)"),
    ("round_not_trunc", "np.trunc(t)", "np.round(t)"),
    ("inverted_scale", "scale = np.float64(nbins) / (hi - lo)", "scale = (hi - lo) / np.float64(nbins)"),
    ("flipped_axis", "t = (v[inside] - lo) * scale", "t = (hi - v[inside]) * scale"),
    ("f32_index_math", "v = np.asarray(v).astype(np.float64)", "v = np.asarray(v).astype(np.float32).astype(np.float64)"),
    ("transposed_flat", "return inside, (iy * nx + ix)[inside]", "return inside, (ix * ny + iy)[inside]"),
    ("axes_swapped", "inx, ix = axis_index(coords[axes[0]]", "inx, ix = axis_index(coords[axes[1]]"),
    ("y_uses_x_bounds", "coords[axes[1]], bounds[2], bounds[3], ny)", "coords[axes[1]], bounds[0], bounds[1], ny)"),
    ("x_only_inside", "inside = inx & iny", "inside = inx"),
    ("min_is_max", "np.minimum.at(kmin, b, keys)", "np.maximum.at(kmin, b, keys)"),
    ("raw_bits_order", "return np.where(bits >= 0, bits, bits ^ _I64_MAX_MAG)\n\n\ndef from",
     "return bits\n\n\ndef from"),
    ("avg_off_by_one", "avg = np.where(empty, np.nan, s / np.maximum(count, 1))",
     "avg = np.where(empty, np.nan, s / np.maximum(count + 1, 1))"),
    ("avg_empty_zero", "avg = np.where(empty, np.nan, s / np.maximum(count, 1))",
     "avg = np.where(empty, 0.0, s / np.maximum(count, 1))"),
    ("sum_of_abs", "s = np.bincount(b, weights=a64, minlength=nb)", "s = np.bincount(b, weights=np.abs(a64), minlength=nb)"),
    ("sum_drops_last", "s = np.bincount(b, weights=a64, minlength=nb)",
     "s = np.bincount(b[:-1], weights=a64[:-1], minlength=nb)"),
    ("attr_f32_rounding", "a64 = np.asarray(a).astype(np.float64)[inside]",
     "a64 = np.asarray(a).astype(np.float32).astype(np.float64)[inside]"),
    ("empty_min_zero", "kmin = np.full(nb, total_order_key(np.array([np.inf]))[0]",
     "kmin = np.full(nb, total_order_key(np.array([0.0]))[0]"),
    ("empty_sum_nan", "s = np.where(empty, 0.0, s)", "s = np.where(empty, np.nan, s)"),
    ("merge_min_is_max", "kmin = np.minimum.reduce(", "kmin = np.maximum.reduce("),
    ("merge_drops_part", 'out = {"count": sum(p["count"] for p in parts)', 'out = {"count": sum(p["count"] for p in parts[1:])'),
]


MUTANTS += [
    ("auto_bounds_keep_nonfinite", "f = v[np.isfinite(v)]", "f = v[~np.isnan(v)]"),
    ("auto_bounds_swapped", 'out += [float(f.min()), float(f.max())] if f.size',
     'out += [float(f.min()), float(f.max()) * (1 + 2**-40)] if f.size'),
    ("zero_scale_unguarded", "    if scale > 0:\n        t = (v[inside] - lo) * scale",
     "    if True:\n        t = (v[inside] - lo) * scale"),
    ("subnormal_extent_kept", "if not (np.isfinite(hi - lo) and np.isfinite(scale)):",
     "if not np.isfinite(hi - lo):"),
]


MUTANTS += [
    ("nd_transposed_flat", "flat += ij * stride", "flat = flat * int(dims[j]) + ij"),
    ("nd_no_stride", "stride *= int(dims[j])", "stride *= 1"),
    ("nd_first_axis_inside", "inside &= inj", "inside = inside if j else inj"),
    ("nd_axis0_bounds", "inj, ij = axis_index(coords[axes[j]], bounds[2 * j], bounds[2 * j + 1], dims[j])",
     "inj, ij = axis_index(coords[axes[j]], bounds[0], bounds[1], dims[j])"),
    ("nd_unreversed_shape", "attrs, tuple(int(v) for v in reversed(dims)))", "attrs, tuple(int(v) for v in dims))"),
    ("nd_axis_column_order", "inj, ij = axis_index(coords[axes[j]]", "inj, ij = axis_index(coords[axes[d - 1 - j]]"),
]


def _mutant_module(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod



@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new):
    mod = _mutant_module(old, new)
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(mod)
        except Exception as e:  # an assertion, or the mutant crashing on a pin
            caught.append((pin.__name__, type(e).__name__))
    assert caught, f"no pin catches the planted mistake {name}"
