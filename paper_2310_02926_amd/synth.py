"""Seeded synthetic particle workloads.

This module only draws inputs. It holds none of the binning arithmetic, so
both the HIP path and the CPU oracle can take their inputs from it.

The paper's workload is particle data from an n-body code (Section 4.1) that
is binned in situ (Section 4.2): columns are variables, rows are particles,
two variables are the mesh axes and the others are reduced per bin.  That data
is not available, so the generators below stand in for it:

* ``uniform_f64``   - uniform positions in [0,1)^2, lognormal(0,1) mass, f64.
* ``gmm_f32``       - a 32-component 2D Gaussian mixture with a fixed share of
  particles outside [0,1]^2, mass plus three velocity components, f32.
* ``hotspot_f32``   - 90% of the particles inside a random 1% of the bins of a
  square grid, the rest uniform, lognormal(0,2) mass, f32.
* ``batch_instances`` - many independent requests of uneven size.
* ``insitu_table``  - ten N-body-like variables binned over nine coordinate
  systems (the multi-grid in situ load of Section 4.3).
* ``halos3d_f32``   - clustered 3-D positions (64 Gaussian halos plus a
  uniform background reaching past the unit cube), lognormal mass, for
  meshes of three axes.

Every generator uses NumPy's PCG64 (``numpy.random.default_rng``) and returns
particles in shuffled order (no spatial locality), columns as separate
contiguous arrays (structure of arrays).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

#: Attribute names in generator order: mass first, then velocity components.
ATTR_NAMES = ("mass", "vx", "vy", "vz")

#: Grid sides used by the batched workload (powers of two from 32 to 1024).
BATCH_SIDES = (32, 64, 128, 256, 512, 1024)

#: Op bit values.  They mirror the C header so that generated requests can be
#: handed to the library directly; the oracle keeps its own copy.
OP_COUNT, OP_SUM, OP_MIN, OP_MAX, OP_AVG = 1, 2, 4, 8, 16
OPS_ALL = 31


@dataclass
class Workload:
    """One binning problem: SoA columns, axes, bounds, grid and ops."""

    coords: List[np.ndarray]
    attrs: List[np.ndarray]
    axes: tuple = (0, 1)
    bounds: tuple = (0.0, 1.0, 0.0, 1.0)
    nx: int = 64
    ny: int = 64
    ops: int = OPS_ALL
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.coords[0].shape[0]) if self.coords else 0

    @property
    def k(self) -> int:
        return len(self.attrs)


def uniform_f64(n: int = 65536, seed: int = 0, nx: int = 64, ny: int = 64) -> Workload:
    """Plain single binning: x, y ~ U[0,1) and mass ~ lognormal(0,1), all f64."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    y = rng.random(n)
    mass = rng.lognormal(0.0, 1.0, n)
    return Workload([x, y], [mass], nx=nx, ny=ny, name=f"uniform_f64_n{n}_{nx}x{ny}")


def _gmm_positions(rng: np.random.Generator, n_in: int, n_out: int, ncomp: int = 32):
    """Positions from an equal-weight isotropic Gaussian mixture, f32.

    ``n_in`` points lie in [0,1)^2 after the cast to f32 (mixture draws are
    rejected and redrawn until they do); ``n_out`` points lie outside the
    closed square [0,1]^2, uniform on [-0.25,1.25)^2 minus that square.
    """
    centres = rng.uniform(0.1, 0.9, size=(ncomp, 2))
    sigmas = rng.uniform(0.01, 0.1, size=ncomp)
    xs = np.empty(n_in + n_out, np.float32)
    ys = np.empty(n_in + n_out, np.float32)
    filled = 0
    while filled < n_in:
        want = n_in - filled
        draw = int(want * 1.3) + 64
        comp = rng.integers(0, ncomp, draw)
        px = (centres[comp, 0] + sigmas[comp] * rng.standard_normal(draw)).astype(np.float32)
        py = (centres[comp, 1] + sigmas[comp] * rng.standard_normal(draw)).astype(np.float32)
        ok = (px >= 0) & (px < 1) & (py >= 0) & (py < 1)
        px, py = px[ok][:want], py[ok][:want]
        xs[filled:filled + px.size] = px
        ys[filled:filled + py.size] = py
        filled += px.size
    filled = 0
    while filled < n_out:
        want = n_out - filled
        draw = int(want * 1.6) + 64
        px = rng.uniform(-0.25, 1.25, draw).astype(np.float32)
        py = rng.uniform(-0.25, 1.25, draw).astype(np.float32)
        inside = (px >= 0) & (px <= 1) & (py >= 0) & (py <= 1)
        px, py = px[~inside][:want], py[~inside][:want]
        xs[n_in + filled:n_in + filled + px.size] = px
        ys[n_in + filled:n_in + filled + py.size] = py
        filled += px.size
    return xs, ys


def gmm_f32(n: int = 1 << 24, seed: int = 0, nx: int = 1024, ny: int = 1024, k: int = 4,
            outside_frac: float = 0.02, ops: int = OPS_ALL) -> Workload:
    """Clustered f32 particles: 32-component Gaussian mixture, a fixed share outside.

    Exactly ``round(outside_frac * n)`` particles lie outside [0,1]^2.
    Attributes (first ``k`` of mass, vx, vy, vz): mass ~ lognormal(0,1),
    velocities ~ N(0,1), all f32.
    """
    rng = np.random.default_rng(seed)
    n_out = int(round(outside_frac * n))
    xs, ys = _gmm_positions(rng, n - n_out, n_out)
    attrs = [rng.lognormal(0.0, 1.0, n).astype(np.float32)]
    for _ in range(1, k):
        attrs.append(rng.standard_normal(n, dtype=np.float32))
    perm = rng.permutation(n)
    return Workload([xs[perm], ys[perm]], [a[perm] for a in attrs[:k]], nx=nx, ny=ny, ops=ops,
                    name=f"gmm_f32_n{n}_{nx}x{ny}_k{k}", meta={"n_outside": n_out})


def hotspot_f32(n: int = 1 << 27, seed: int = 0, side: int = 2048, hot_frac: float = 0.9,
                hot_bins_frac: float = 0.01, contiguous: bool = False) -> Workload:
    """Hot-spot f32 particles on a ``side`` x ``side`` grid over [0,1]^2.

    A hot set H of floor(hot_bins_frac * side^2) bins is drawn without
    replacement (or, with ``contiguous``, taken as a square block).
    round(hot_frac * n) particles go to a bin drawn uniformly from H, at
    ((ix+u)/side, (iy+v)/side) with u, v ~ U(0.05, 0.95), computed in f64 and
    then cast to f32 (the 0.05 margin keeps every such point inside its bin).
    The remaining particles are uniform on [0,1)^2.  mass ~ lognormal(0,2), f32.
    """
    rng = np.random.default_rng(seed)
    nbins = side * side
    nhot_bins = int(hot_bins_frac * nbins)
    if contiguous:
        s = int(np.ceil(np.sqrt(nhot_bins)))
        x0 = int(rng.integers(0, side - s))
        y0 = int(rng.integers(0, side - s))
        yy, xx = np.meshgrid(np.arange(y0, y0 + s), np.arange(x0, x0 + s), indexing="ij")
        hot = (yy * side + xx).ravel()[:nhot_bins]
    else:
        hot = rng.choice(nbins, size=nhot_bins, replace=False)
    n_hot = int(round(hot_frac * n))
    pick = hot[rng.integers(0, nhot_bins, n_hot)]
    ix = pick % side
    iy = pick // side
    u = rng.uniform(0.05, 0.95, n_hot)
    v = rng.uniform(0.05, 0.95, n_hot)
    x = np.empty(n, np.float32)
    y = np.empty(n, np.float32)
    x[:n_hot] = ((ix + u) / side).astype(np.float32)
    y[:n_hot] = ((iy + v) / side).astype(np.float32)
    del ix, iy, u, v, pick
    x[n_hot:] = rng.random(n - n_hot, dtype=np.float32)
    y[n_hot:] = rng.random(n - n_hot, dtype=np.float32)
    mass = rng.lognormal(0.0, 2.0, n).astype(np.float32)
    perm = rng.permutation(n)
    x = x[perm]
    y = y[perm]
    del perm
    return Workload([x, y], [mass], nx=side, ny=side,
                    name=f"hotspot_f32_n{n}_{side}x{side}",
                    meta={"hot_bins": np.sort(hot), "n_hot": n_hot})


def halos3d_f32(n: int = 1 << 26, seed: int = 0, side: int = 128, halo_frac: float = 0.8,
                nhalo: int = 64) -> Workload:
    """Clustered 3-D f32 positions for a ``side``^3 mesh over [0,1]^3.

    round(halo_frac * n) particles belong to one of ``nhalo`` equal-weight
    isotropic Gaussian halos (centres U(0.1,0.9)^3, sigma U(0.01,0.08));
    the rest are uniform on [-0.05,1.05)^3, so some fall outside the mesh
    (as do halo particles in the tails).  mass ~ lognormal(0,1).  Columns:
    x, y, z; axes (0, 1, 2) in ``meta["nd"]`` with bounds and dims."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.1, 0.9, size=(nhalo, 3))
    sigmas = rng.uniform(0.01, 0.08, size=nhalo)
    n_halo = int(round(halo_frac * n))
    comp = rng.integers(0, nhalo, n_halo)
    cols = []
    for d in range(3):
        c = np.empty(n, np.float32)
        c[:n_halo] = (centres[comp, d] + sigmas[comp] * rng.standard_normal(n_halo, dtype=np.float32))
        c[n_halo:] = rng.uniform(-0.05, 1.05, n - n_halo).astype(np.float32)
        cols.append(c)
    del comp
    mass = rng.lognormal(0.0, 1.0, n).astype(np.float32)
    perm = rng.permutation(n)
    cols = [c[perm] for c in cols]
    mass = mass[perm]
    return Workload(cols, [mass], axes=(0, 1), bounds=(0.0, 1.0, 0.0, 1.0), nx=side, ny=side * side,
                    name=f"halos3d_f32_n{n}_{side}cube",
                    meta={"nd": ((0, 1, 2), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), (side, side, side))})


def random_ops(rng: np.random.Generator) -> int:
    """Each of the five ops with probability 1/2, redrawn if the set is empty."""
    while True:
        ops = 0
        for bit in (OP_COUNT, OP_SUM, OP_MIN, OP_MAX, OP_AVG):
            if rng.random() < 0.5:
                ops |= bit
        if ops:
            return ops


@dataclass
class InstanceSpec:
    n: int
    side: int
    k: int
    ops: int
    seed: int


def batch_specs(count: int = 256, seed: int = 0, n_lo: float = 1e3, n_hi: float = 1e7,
                sides: Sequence[int] = BATCH_SIDES) -> List[InstanceSpec]:
    """Shapes of the batched workload: n log-uniform in [n_lo, n_hi], square
    grids with a side from ``sides``, 1-4 attributes, a random op set."""
    rng = np.random.default_rng(seed)
    seeds = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i in range(count):
        n = int(round(10 ** rng.uniform(np.log10(n_lo), np.log10(n_hi))))
        side = int(sides[int(rng.integers(0, len(sides)))])
        k = int(rng.integers(1, 5))
        ops = random_ops(rng)
        out.append(InstanceSpec(n, side, k, ops, int(seeds[i].generate_state(1)[0])))
    return out


def instance(spec: InstanceSpec) -> Workload:
    """Particles for one batched request: the clustered generator at the spec's shape."""
    return gmm_f32(n=spec.n, seed=spec.seed, nx=spec.side, ny=spec.side, k=spec.k, ops=spec.ops)


def batch_instances(count: int = 256, seed: int = 0, **kw) -> List[Workload]:
    return [instance(s) for s in batch_specs(count, seed, **kw)]


def poisson_arrivals(rate: float, count: int, seed: int = 0) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def edge_points(lo: float, hi: float, nbins: int, dtype=np.float64) -> np.ndarray:
    """Adversarial coordinates: every bin edge, its neighbours one ulp away,
    the bounds themselves, and values outside, NaN and +-Inf."""
    dt = np.dtype(dtype)
    edges = lo + (hi - lo) * np.arange(nbins + 1, dtype=np.float64) / nbins
    e = edges.astype(dt)
    pts = [e, np.nextafter(e, dt.type(-np.inf)), np.nextafter(e, dt.type(np.inf)),
           np.array([lo, hi, np.nan, np.inf, -np.inf, lo - (hi - lo), hi + (hi - lo)], dtype=dt)]
    return np.concatenate(pts).astype(dt)


# Columns of the in situ table and the coordinate systems binned over it.
INSITU_COLUMNS = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "m")
INSITU_PLANES = ((0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5), (6, 7), (6, 8), (7, 8))


@dataclass
class InsituTable:
    columns: List[np.ndarray]
    planes: Sequence[tuple]
    bounds: List[tuple]
    n: int


def insitu_table(n: int = 1 << 20, seed: int = 0, dtype=np.float32) -> InsituTable:
    """An N-body-like particle table for the multi-grid in situ load: ten
    variables (position uniform in [-1,1)^3, velocity and acceleration
    N(0,1) per component, mass lognormal(0,1)) binned over nine coordinate
    systems: the three planes of position, of velocity and of acceleration.
    Bounds: [-1,1] for positions, [-4,4] for the other planes (particles
    beyond 4 sigma fall outside)."""
    rng = np.random.default_rng(seed)
    cols = [rng.uniform(-1.0, 1.0, n).astype(dtype) for _ in range(3)]
    cols += [rng.standard_normal(n).astype(dtype) for _ in range(6)]
    cols.append(rng.lognormal(0.0, 1.0, n).astype(dtype))
    bounds = []
    for a, b in INSITU_PLANES:
        lo, hi = (-1.0, 1.0) if a < 3 else (-4.0, 4.0)
        bounds.append((lo, hi, lo, hi))
    return InsituTable(cols, INSITU_PLANES, bounds, n)
